// knn_rerank_backward.hip -- FP32 rescoring of low-precision candidates, and the
// backward pass through the retrieved scores.
//
// Rerank: the distance kernel ranks bins with BF16 or FP8 products; the best Kr
// bin winners are rescored here in FP32 from the caller's original rows, one wave
// per query (16-lane groups per candidate, a fixed butterfly sums the pieces), and
// the best K by (score, lower index) are kept with a register bitonic sort.
//
// Backward: with the selection held fixed, d score(q_i, x_j) is a gather over the
// selected rows for dQ (one wave per query) and a scatter-add into dX (one wave
// per selected (query, row) pair, FP32 atomics).
#include "knn_common.cuh"

namespace knn {

namespace {

constexpr int kRerankThreads = 256;  // 4 waves, one query each
constexpr int kRerankMaxKr = 1024;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wave per query.  Candidate scores: groups of 16 lanes each take a candidate
// row and split its depth into 16-byte pieces (4 FP32 or 8 BF16 elements per lane
// per pass); a fixed 16-lane butterfly sums the pieces.  Keys (score, lower index
// first on ties) go through the wave's LDS slots into a register bitonic sort.
// XDT: the original rows' type (FP32 or BF16), fixed per instance so that an FP32
// instance holds 4 query elements per piece, not 8
template <int R, int XDT>
__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(const int32_t* __restrict__ cand, int64_t M, int Kr,
                                                                const void* __restrict__ Q, int q_dt,
                                                                const void* __restrict__ X, int D,
                                                                int metric, const float* __restrict__ x_half_norm,
                                                                const float* __restrict__ x_rnorm, int K,
                                                                float* __restrict__ out_val,
                                                                int32_t* __restrict__ out_idx) {
  __shared__ unsigned long long slots[kRerankThreads / 64][64 * R];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane >> 4, gl = lane & 15;
  constexpr int E = XDT == DT_F32 ? 4 : 8;  // elements per 16-byte piece
  const int per_pass = 16 * E;
  const int passes = (D + per_pass - 1) / per_pass;  // <= 4 for D <= 256
  // whole 16-byte pieces when every row starts 16-byte aligned
  const bool vec = (reinterpret_cast<uintptr_t>(X) & 15) == 0 && (D % E) == 0;
  unsigned long long* key_slot = slots[wave];
  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < M; i += (int64_t)gridDim.x * 4) {
    // this lane's query elements, in the order its pieces cover the depth
    float q[4][E];
#pragma unroll
    for (int ps = 0; ps < 4; ++ps)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int d = ps * per_pass + gl * E + e;
        q[ps][e] = (ps < passes && d < D) ? load_elem(Q, q_dt, i * D + d) : 0.f;
      }
    float rq = 1.f;
    if (metric == MET_COSINE) {
      float qq = 0.f;
      for (int d = lane; d < D; d += 64) {
        const float v = load_elem(Q, q_dt, i * D + d);
        qq = fmaf(v, v, qq);
      }
      qq = wave_sum(qq);
      rq = qq > 0.f ? 1.f / sqrtf(qq) : 0.f;
    }
    for (int c0 = 0; c0 < 64 * R; c0 += 4) {
      const int c = c0 + grp;
      unsigned long long key = 0ull;  // below every real key: pads sort last
      if (c0 < Kr) {
        const int j = c < Kr ? cand[i * Kr + c] : -1;
        float dot = 0.f;
        if (j >= 0) {
#pragma unroll
          for (int ps = 0; ps < 4; ++ps) {
            if (ps >= passes) break;
            const int d0 = ps * per_pass + gl * E;
            if (d0 < D) {
              if constexpr (XDT == DT_F32) {
                const float* xr = reinterpret_cast<const float*>(X) + (int64_t)j * D + d0;
                if (vec) {
                  const float4 v = *reinterpret_cast<const float4*>(xr);
                  dot = fmaf(q[ps][0], v.x, dot);
                  dot = fmaf(q[ps][1], v.y, dot);
                  dot = fmaf(q[ps][2], v.z, dot);
                  dot = fmaf(q[ps][3], v.w, dot);
                } else {
                  for (int e = 0; e < 4 && d0 + e < D; ++e) dot = fmaf(q[ps][e], xr[e], dot);
                }
              } else {
                const unsigned short* xr = reinterpret_cast<const unsigned short*>(X) + (int64_t)j * D + d0;
                if (vec) {
                  const u32x4 v = *reinterpret_cast<const u32x4*>(xr);
#pragma unroll
                  for (int w = 0; w < 4; ++w) {
                    dot = fmaf(q[ps][2 * w], __uint_as_float(v[w] << 16), dot);
                    dot = fmaf(q[ps][2 * w + 1], __uint_as_float(v[w] & 0xFFFF0000u), dot);
                  }
                } else {
                  for (int e = 0; e < 8 && d0 + e < D; ++e) dot = fmaf(q[ps][e], __uint_as_float((unsigned)xr[e] << 16), dot);
                }
              }
            }
          }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 16);
        float sc = dot;
        if (metric == MET_L2) sc = dot - (j >= 0 ? x_half_norm[j] : 0.f);
        if (metric == MET_COSINE) sc = dot * rq * (j >= 0 ? x_rnorm[j] : 0.f);
        if (j < 0) sc = -INFINITY;
        key = c < Kr ? (((unsigned long long)float_key(sc) << 32) | (unsigned)~(unsigned)j) : 0ull;
      }
      if (gl == 0) key_slot[c] = key;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long k[R];
#pragma unroll
    for (int r = 0; r < R; ++r) k[r] = key_slot[64 * r + lane];
    wave_sort_desc<R>(k, lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = 64 * r + lane;
      if (e < K) {
        const float v = key_float((unsigned)(k[r] >> 32));
        out_val[i * K + e] = metric == MET_L2 ? -v : v;
        out_idx[i * K + e] = (int32_t)~(unsigned)(k[r] & 0xFFFFFFFFull);
      }
    }
    // the next query rewrites this wave's slots: finish the reads first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
  const int64_t want = ceil_div(M, 4);
  const unsigned grid = (unsigned)(want < 16384 ? want : 16384);
#define KNN_RERANK(R_)                                                                                        \
  do {                                                                                                        \
    if (x_dt == DT_F32)                                                                                       \
      rerank_kernel<R_, DT_F32><<<grid, kRerankThreads, 0, s>>>(cand, M, Kr, Q, q_dt, X, D, metric, x_half_norm, \
                                                                x_rnorm, K, out_val, out_idx);                  \
    else                                                                                                      \
      rerank_kernel<R_, DT_BF16><<<grid, kRerankThreads, 0, s>>>(cand, M, Kr, Q, q_dt, X, D, metric,            \
                                                                 x_half_norm, x_rnorm, K, out_val, out_idx);    \
  } while (0)
  if (Kr <= 64)
    KNN_RERANK(1);
  else if (Kr <= 128)
    KNN_RERANK(2);
  else if (Kr <= 256)
    KNN_RERANK(4);
  else if (Kr <= 512)
    KNN_RERANK(8);
  else
    KNN_RERANK(16);
#undef KNN_RERANK
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
