// knn_select.hip -- exact top-K over candidate lists (the ExactRescoring step, Sec. 5).
//
// The paper sorts the M x L bin winners with a bitonic sort and truncates to K
// (O(M L log^2 L)).  Here each row gets one workgroup running an MSB-first radix
// select on order-preserving 32-bit keys of the scores (4 passes of 8 bits over
// the row, a 256-bin LDS histogram and a one-wave scan per pass) to find the K-th
// best score T exactly; if T is shared by more rows than are still needed, a
// second radix select on the row indices keeps the lowest ones.  The K survivors
// are then bitonic-sorted in LDS by (score, lower index first) and written best
// first.  Cost per row: O(L) reads per pass instead of O(L log^2 L).  Rows of at
// most 1024 candidates instead take one wave each and a register bitonic sort.
// Candidates may still be 4-row group codes; they keep their code (resolved
// afterwards).
#include "knn_common.cuh"

namespace knn {

namespace {

constexpr int kSelThreads = 256;
constexpr int kMaxK = 1024;

// Scores are keyed by float_key(sgn * v + 0): adding +0 turns -0 into +0, so the two
// zeros tie as they do under the strict comparison of the bin reduce.
// Candidate indices are rows (>= 0), 4-row group codes (-2 - start/4, resolved
// later) or -1 (none).  The tie-break key orders them by row: unit u = 2*start +
// is_group is unique per candidate (bins are disjoint), and the sort uses ~u so
// that a lower row ranks first; "none" maps to 0, below every real unit.
__device__ __forceinline__ unsigned unit_lo(int32_t code) {
  if (code >= 0) return ~(2u * (unsigned)code);
  if (code == -1) return 0u;
  return ~(2u * 4u * (unsigned)(-2 - code) + 1u);
}
__device__ __forceinline__ int32_t unit_code(unsigned lo) {
  if (lo == 0u) return -1;
  const unsigned u = ~lo;
  return (u & 1u) ? -2 - (int32_t)(u >> 3) : (int32_t)(u >> 1);
}

struct SelShared {
  unsigned hist[256];
  unsigned long long keys[kMaxK];
  int digit, krem, eqcount, count;
};

// one radix pass: histogram of byte `shift` of key(c) over candidates whose key
// matches prefix under mask; returns the digit holding the krem-th largest and
// updates krem to the rank inside that digit
template <class KeyFn>
__device__ __forceinline__ void radix_pass(SelShared& sh, int64_t n, KeyFn key, unsigned prefix, unsigned mask,
                                           int shift, int& krem, unsigned& digit, int& eqcount) {
  const int tid = threadIdx.x;
  for (int i = tid; i < 256; i += kSelThreads) sh.hist[i] = 0;
  __syncthreads();
  for (int64_t c = tid; c < n; c += kSelThreads) {
    bool ok;
    unsigned k = key(c, ok);
    if (ok && (k & mask) == prefix) atomicAdd(&sh.hist[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (tid < 64) {
    const int l = tid;
    unsigned cnt[4];
    unsigned sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cnt[j] = sh.hist[255 - 4 * l - j];
      sum += cnt[j];
    }
    unsigned incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      unsigned t = __shfl_up(incl, off);
      if (l >= off) incl += t;
    }
    const unsigned excl = incl - sum;
    if (excl < (unsigned)krem && (unsigned)krem <= incl) {
      unsigned acc = excl;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (acc + cnt[j] >= (unsigned)krem) {
          sh.digit = 255 - 4 * l - j;
          sh.krem = krem - (int)acc;
          sh.eqcount = (int)cnt[j];
          break;
        }
        acc += cnt[j];
      }
    }
  }
  __syncthreads();
  digit = (unsigned)sh.digit;
  krem = sh.krem;
  eqcount = sh.eqcount;
}

// candidate c of the row is V[c * es], A[c * es]; output e goes to out_*[e * eo]
__device__ void select_row(SelShared& sh, const float* __restrict__ V, const int32_t* __restrict__ A, int64_t n,
                           int64_t es, int K, bool minimize, float* __restrict__ out_val,
                           int32_t* __restrict__ out_idx, int64_t eo) {
  const int tid = threadIdx.x;
  if (K > n) K = (int)n;
  const float sgn = minimize ? -1.f : 1.f;  // rank by sgn * value, larger first
  // phase 1: K-th best score key
  unsigned prefix = 0, mask = 0, digit = 0;
  int krem = K, eqcount = 0;
  auto vkey = [&](int64_t c, bool& ok) {
    ok = true;
    return float_key(sgn * V[c * es] + 0.f);
  };
  for (int shift = 24; shift >= 0; shift -= 8) {
    radix_pass(sh, n, vkey, prefix, mask, shift, krem, digit, eqcount);
    prefix |= digit << shift;
    mask |= 255u << shift;
  }
  const unsigned T = prefix;
  // phase 2: among score == T keep the krem lowest row indices
  unsigned T2 = 0;  // threshold on ~index (larger = lower index)
  const bool all_eq = (eqcount == krem);
  if (!all_eq) {
    unsigned p2 = 0, m2 = 0, d2 = 0;
    int kr2 = krem, eq2 = 0;
    auto ikey = [&](int64_t c, bool& ok) {
      ok = float_key(sgn * V[c * es] + 0.f) == T;
      return unit_lo(A[c * es]);
    };
    for (int shift = 24; shift >= 0; shift -= 8) {
      radix_pass(sh, n, ikey, p2, m2, shift, kr2, d2, eq2);
      p2 |= d2 << shift;
      m2 |= 255u << shift;
    }
    T2 = p2;
  }
  // phase 3: collect the K winners
  if (tid == 0) sh.count = 0;
  __syncthreads();
  for (int64_t c = tid; c < n; c += kSelThreads) {
    const unsigned k = float_key(sgn * V[c * es] + 0.f);
    const unsigned lo = unit_lo(A[c * es]);
    const bool take = (k > T) || (k == T && (all_eq || lo >= T2));
    if (take) {
      int pos = atomicAdd(&sh.count, 1);
      if (pos < K) sh.keys[pos] = ((unsigned long long)k << 32) | lo;
    }
  }
  __syncthreads();
  int kp = 1;
  while (kp < K) kp <<= 1;
  for (int i = K + tid; i < kp; i += kSelThreads) sh.keys[i] = 0ull;
  __syncthreads();
  // phase 4: bitonic sort, descending
  for (int size = 2; size <= kp; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < kp; i += kSelThreads) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          unsigned long long a = sh.keys[i], b = sh.keys[j];
          if (desc ? (a < b) : (a > b)) {
            sh.keys[i] = b;
            sh.keys[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < K; i += kSelThreads) {
    const unsigned long long key = sh.keys[i];
    float v = key_float((unsigned)(key >> 32));
    out_val[i * eo] = sgn * v;
    out_idx[i * eo] = unit_code((unsigned)(key & 0xFFFFFFFFull));
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSelThreads) void select_kernel(const float* __restrict__ V,
                                                             const int32_t* __restrict__ A, int64_t rows, int64_t n,
                                                             int64_t ldv, int64_t es, int K, int minimize,
                                                             float* __restrict__ out_val,
                                                             int32_t* __restrict__ out_idx, int64_t ldout,
                                                             int64_t eo) {
  __shared__ SelShared sh;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
    select_row(sh, V + r * ldv, A + r * ldv, n, es, K, minimize != 0, out_val + r * ldout, out_idx + r * ldout,
               eo);
}

__global__ __launch_bounds__(kSelThreads) void select_rows_kernel(const SelRow* __restrict__ rows_desc,
                                                                  int64_t rows) {
  __shared__ SelShared sh;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const SelRow d = rows_desc[r];
    select_row(sh, d.V, d.A, d.n, 1, d.K, d.minimize != 0, d.out_val, d.out_idx, 1);
  }
}

// Rows of at most 64*R candidates: one wave per row, keys (score, then lower unit)
// held in registers and sorted by a bitonic network of shuffles; no LDS, no
// workgroup barriers.  Same order as the radix path.
template <int R>
__global__ __launch_bounds__(256) void select_wave_kernel(const float* __restrict__ V, const int32_t* __restrict__ A,
                                                          int64_t rows, int n, int64_t ldv, int64_t es, int K,
                                                          int minimize, float* __restrict__ out_val,
                                                          int32_t* __restrict__ out_idx, int64_t ldout, int64_t eo) {
  const int lane = threadIdx.x & 63;
  const float sgn = minimize ? -1.f : 1.f;
  if (K > n) K = n;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gridDim.x * 4) {
    unsigned long long k[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int c = 64 * i + lane;
      k[i] = c < n ? (((unsigned long long)float_key(sgn * V[r * ldv + c * es] + 0.f) << 32) |
                      unit_lo(A[r * ldv + c * es]))
                   : 0ull;
    }
    wave_sort_desc<R>(k, lane);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = 64 * i + lane;
      if (e < K) {
        out_val[r * ldout + e * eo] = sgn * key_float((unsigned)(k[i] >> 32));
        out_idx[r * ldout + e * eo] = unit_code((unsigned)(k[i] & 0xFFFFFFFFull));
      }
    }
  }
}

}  // namespace

hipError_t launch_select(const float* V, const int32_t* A, int64_t rows, int64_t n, int64_t ldv, int K,
                         bool minimize, float* out_val, int32_t* out_idx, int64_t ldout, hipStream_t s, int64_t es,
                         int64_t eo) {
  (void)hipGetLastError();  // report only this call's launch errors
  if (rows == 0) return hipSuccess;
  if (K > kMaxK || K < 1 || n < 1) return hipErrorInvalidValue;
  if (n <= 1024) {  // short rows: a wave per row, sorted in registers
    const int64_t want = ceil_div(rows, 4);
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    const int nn = (int)n, mz = minimize ? 1 : 0;
#define KNN_SELW(R_) \
  select_wave_kernel<R_><<<grid, 256, 0, s>>>(V, A, rows, nn, ldv, es, K, mz, out_val, out_idx, ldout, eo)
    if (n <= 64)
      KNN_SELW(1);
    else if (n <= 128)
      KNN_SELW(2);
    else if (n <= 256)
      KNN_SELW(4);
    else if (n <= 512)
      KNN_SELW(8);
    else
      KNN_SELW(16);
#undef KNN_SELW
    return hipGetLastError();
  }
  const int64_t grid = rows < 65536 ? rows : 65536;
  select_kernel<<<(unsigned)grid, kSelThreads, 0, s>>>(V, A, rows, n, ldv, es, K, minimize ? 1 : 0, out_val,
                                                       out_idx, ldout, eo);
  return hipGetLastError();
}

hipError_t launch_select_rows(const SelRow* d_rows, int64_t rows, int max_K, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  if (rows == 0) return hipSuccess;
  if (max_K > kMaxK) return hipErrorInvalidValue;
  const int64_t grid = rows < 65536 ? rows : 65536;
  select_rows_kernel<<<(unsigned)grid, kSelThreads, 0, s>>>(d_rows, rows);
  return hipGetLastError();
}

}  // namespace knn
