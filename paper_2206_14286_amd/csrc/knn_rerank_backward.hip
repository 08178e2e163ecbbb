// knn_rerank_backward.hip -- FP32 rescoring of low-precision candidates, and the
// backward pass through the retrieved scores.
//
// Rerank: the distance kernel ranks bins with BF16 or FP8 products; the best Kr
// bin winners are rescored here in FP32 from the caller's original rows, one
// workgroup per query (lanes split the depth, a fixed butterfly sums the lanes),
// and the best K by (score, lower index) are kept with an LDS bitonic sort.
//
// Backward: with the selection held fixed, d score(q_i, x_j) is a gather over the
// selected rows for dQ (one wave per query) and a scatter-add into dX (one wave
// per selected (query, row) pair, FP32 atomics).
#include "knn_common.cuh"

namespace knn {

namespace {

constexpr int kRerankThreads = 256;
constexpr int kRerankMaxKr = 1024;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(const int32_t* __restrict__ cand, int64_t M, int Kr,
                                                                const void* __restrict__ Q, int q_dt,
                                                                const void* __restrict__ X, int x_dt, int D,
                                                                int metric, const float* __restrict__ x_half_norm,
                                                                const float* __restrict__ x_rnorm, int K,
                                                                float* __restrict__ out_val,
                                                                int32_t* __restrict__ out_idx) {
  __shared__ unsigned long long keys[kRerankMaxKr];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int kp = 1;
  while (kp < Kr) kp <<= 1;
  for (int64_t i = blockIdx.x; i < M; i += gridDim.x) {
    float q[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int d = lane + 64 * s;
      q[s] = d < D ? load_elem(Q, q_dt, i * D + d) : 0.f;
    }
    float rq = 1.f;
    if (metric == MET_COSINE) {
      float qq = 0.f;
#pragma unroll
      for (int s = 0; s < 4; ++s) qq = fmaf(q[s], q[s], qq);
      qq = wave_sum(qq);
      rq = qq > 0.f ? 1.f / sqrtf(qq) : 0.f;
    }
    for (int c = wave; c < kp; c += 4) {
      unsigned long long key = 0ull;
      if (c < Kr) {
        const int j = cand[i * Kr + c];
        float dot = 0.f;
        if (j >= 0) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int d = lane + 64 * s;
            if (d < D) dot = fmaf(q[s], load_elem(X, x_dt, (int64_t)j * D + d), dot);
          }
        }
        dot = wave_sum(dot);
        float sc = dot;
        if (metric == MET_L2) sc = dot - (j >= 0 ? x_half_norm[j] : 0.f);
        if (metric == MET_COSINE) sc = dot * rq * (j >= 0 ? x_rnorm[j] : 0.f);
        if (j < 0) sc = -INFINITY;
        key = ((unsigned long long)float_key(sc) << 32) | (unsigned)~(unsigned)j;
      }
      if (lane == 0) keys[c] = key;
    }
    __syncthreads();
    for (int size = 2; size <= kp; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int a = tid; a < kp; a += kRerankThreads) {
          const int b = a ^ stride;
          if (b > a) {
            const bool desc = (a & size) == 0;
            unsigned long long x = keys[a], y = keys[b];
            if (desc ? (x < y) : (x > y)) {
              keys[a] = y;
              keys[b] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int k = tid; k < K; k += kRerankThreads) {
      const unsigned long long key = keys[k];
      const float v = key_float((unsigned)(key >> 32));
      out_val[i * K + k] = metric == MET_L2 ? -v : v;
      out_idx[i * K + k] = (int32_t)~(unsigned)(key & 0xFFFFFFFFull);
    }
    __syncthreads();
  }
}

// one wave per query: dQ_i = sum_k g_ik d score/d q
__global__ __launch_bounds__(256) void backward_dq_kernel(const float* __restrict__ g, const int32_t* __restrict__ idx,
                                                          const void* __restrict__ Q, const void* __restrict__ X,
                                                          int dt, int64_t M, int64_t N, int D, int K, int metric,
                                                          float* __restrict__ dQ) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;
  float q[4], acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int d = lane + 64 * s;
    q[s] = d < D ? load_elem(Q, dt, i * D + d) : 0.f;
  }
  float qq = 0.f;
  if (metric == MET_COSINE) {
#pragma unroll
    for (int s = 0; s < 4; ++s) qq = fmaf(q[s], q[s], qq);
    qq = wave_sum(qq);
  }
  for (int k = 0; k < K; ++k) {
    const int32_t j = idx[i * K + k];
    if (j < 0 || j >= N) continue;
    const float gk = g[i * K + k];
    float x[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int d = lane + 64 * s;
      x[s] = d < D ? load_elem(X, dt, (int64_t)j * D + d) : 0.f;
    }
    if (metric == MET_MIPS) {
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = fmaf(gk, x[s], acc[s]);
    } else if (metric == MET_L2) {
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = fmaf(-gk, x[s], acc[s]);
    } else {
      float xx = 0.f, dot = 0.f;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        xx = fmaf(x[s], x[s], xx);
        dot = fmaf(q[s], x[s], dot);
      }
      xx = wave_sum(xx);
      dot = wave_sum(dot);
      if (qq > 0.f && xx > 0.f) {
        const float nqx = sqrtf(qq) * sqrtf(xx);
        const float c = dot / nqx;
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s] += gk * (x[s] / nqx - c * q[s] / qq);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int d = lane + 64 * s;
    if (d < D) dQ[i * D + d] = acc[s];
  }
}

// one wave per selected (query, row) pair: dX_j += g_ik d score/d x
__global__ __launch_bounds__(256) void backward_dx_kernel(const float* __restrict__ g, const int32_t* __restrict__ idx,
                                                          const void* __restrict__ Q, const void* __restrict__ X,
                                                          int dt, int64_t M, int64_t N, int D, int K, int metric,
                                                          float* __restrict__ dX) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= M * K) return;
  const int64_t i = p / K;
  const int32_t j = idx[p];
  if (j < 0 || j >= N) return;
  const float gk = g[p];
  float q[4], x[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int d = lane + 64 * s;
    q[s] = d < D ? load_elem(Q, dt, i * D + d) : 0.f;
    x[s] = (d < D && metric != MET_MIPS) ? load_elem(X, dt, (int64_t)j * D + d) : 0.f;
  }
  float coef_q = gk, coef_x = 0.f;
  if (metric == MET_L2) {
    coef_q = -gk;
    coef_x = gk;
  } else if (metric == MET_COSINE) {
    float qq = 0.f, xx = 0.f, dot = 0.f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      qq = fmaf(q[s], q[s], qq);
      xx = fmaf(x[s], x[s], xx);
      dot = fmaf(q[s], x[s], dot);
    }
    qq = wave_sum(qq);
    xx = wave_sum(xx);
    dot = wave_sum(dot);
    if (!(qq > 0.f && xx > 0.f)) return;
    const float nqx = sqrtf(qq) * sqrtf(xx);
    coef_q = gk / nqx;
    coef_x = -gk * (dot / nqx) / xx;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int d = lane + 64 * s;
    if (d < D) atomicAdd(&dX[(int64_t)j * D + d], coef_q * q[s] + coef_x * x[s]);
  }
}

}  // namespace

hipError_t launch_rerank(const int32_t* cand, int64_t M, int Kr, const void* Q, int q_dt, const void* X, int x_dt,
                         int D, int metric, const float* x_half_norm, const float* x_rnorm, int K, float* out_val,
                         int32_t* out_idx, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  if (M == 0) return hipSuccess;
  if (Kr > kRerankMaxKr || K > Kr || D > 256) return hipErrorInvalidValue;
  const int64_t grid = M < 65536 ? M : 65536;
  rerank_kernel<<<(unsigned)grid, kRerankThreads, 0, s>>>(cand, M, Kr, Q, q_dt, X, x_dt, D, metric, x_half_norm,
                                                          x_rnorm, K, out_val, out_idx);
  return hipGetLastError();
}

hipError_t launch_backward(const float* g, const int32_t* idx, const void* Q, const void* X, int dt, int64_t M,
                           int64_t N, int D, int K, int metric, float* dQ, float* dX, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  if (M == 0) return hipSuccess;
  if (D > 256) return hipErrorInvalidValue;
  if (dQ) {
    backward_dq_kernel<<<(unsigned)ceil_div(M, 4), 256, 0, s>>>(g, idx, Q, X, dt, M, N, D, K, metric, dQ);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (dX) {
    backward_dx_kernel<<<(unsigned)ceil_div(M * K, 4), 256, 0, s>>>(g, idx, Q, X, dt, M, N, D, K, metric, dX);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace knn
