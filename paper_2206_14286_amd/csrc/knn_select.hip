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
// Candidate indices are rows (>= 0), codes of rows still to be resolved (groups
// -2 - s/4, pairs -2 - 2^29 - s/4, quads -2 - 2^30 - s/16 for a first row s; see the
// distance kernel) or -1 (none).  The tie-break key orders them by first row: the unit
// u = 2 s (+1 group, +3 pair, +5 quad) is unique per candidate (bins are disjoint), and
// the sort uses ~u so that a lower row ranks first; "none" maps to 0, below every
// real unit.
__device__ __forceinline__ unsigned unit_lo(int32_t code) {
  if (code >= 0) return ~(2u * (unsigned)code);
  if (code == -1) return 0u;
  if (code > -2 - (1 << 29)) return ~(8u * (unsigned)(-2 - code) + 1u);
  if (code > -2 - (1 << 30)) return ~(8u * (unsigned)(-2 - (1 << 29) - code) + 3u);
  return ~(32u * (unsigned)(-2 - (1 << 30) - code) + 5u);
}
__device__ __forceinline__ int32_t unit_code(unsigned lo) {
  if (lo == 0u) return -1;
  const unsigned u = ~lo;
  if (!(u & 1u)) return (int32_t)(u >> 1);
  if ((u & 7u) == 1u) return -2 - (int32_t)(u >> 3);
  if ((u & 7u) == 3u) return -2 - (1 << 29) - (int32_t)(u >> 3);
  return -2 - (1 << 30) - (int32_t)(u >> 5);
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

// Rows of many candidates: the K-th best key is found from a histogram over the row's
// own key range instead of byte by byte.  Pass 1: the smallest and largest key of the
// row.  Pass 2: a kRangeBuckets-bucket histogram of (key - kmin) >> shift, shift the
// smallest that fits the range into the buckets; the bucket b* holding the K-th best is
// found by a scan from the top.  Pass 3: candidates in buckets above b* are winners;
// those in b* are collected in LDS and sorted by (key, lower index first), and the best
// of them complete the K.  Three reads of the row instead of five or more; when b*
// holds more than kRangeCap candidates (a dense cluster of equal-looking scores) the
// row falls back to the byte-wise radix select.
// Sized for occupancy: 16 KB of LDS and <= 64 VGPRs give eight workgroups per CU, which
// the passes (latency-bound: each wave waits on its loads) need more than finer buckets
// or more loads in flight per thread (cosine FP8, 10,000 rows of 18,750: 2048 buckets, a
// 2048-key tie buffer, 8 loads per thread at 4 waves/SIMD 3.72 ms per search; these
// settings 3.40 ms).
constexpr int kRangeBuckets = 1024;
constexpr int kRangeCap = 512;

struct RangeShared {
  unsigned hist[kRangeBuckets];
  unsigned long long bnd[kRangeCap];
  unsigned kmin_w[kSelThreads / 64], kmax_w[kSelThreads / 64];
  int bstar, above, nb, nhi;
};

union SelUnion {
  SelShared radix;
  struct {
    unsigned long long keys[kMaxK];
    RangeShared r;
  } range;
};

__device__ __forceinline__ void bitonic_desc_lds(unsigned long long* a, int m) {
  // m a power of two; all threads of the block take part
  for (int size = 2; size <= m; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < m; i += kSelThreads) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const unsigned long long x = a[i], y = a[j];
          if (desc ? (x < y) : (x > y)) {
            a[i] = y;
            a[j] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

// f(c, key) for every candidate c of the row, the keys of kSelThreads * 4 candidates
// loaded before any is used (more per thread costs registers and occupancy: 8 and 16
// were slower)
template <class F>
__device__ __forceinline__ void for_each_key(const float* __restrict__ V, int64_t n, int64_t es, float sgn, F f) {
  constexpr int U = 4;
  for (int64_t c0 = threadIdx.x; c0 < n; c0 += (int64_t)kSelThreads * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = c0 + (int64_t)u * kSelThreads;
      v[u] = c < n ? V[c * es] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = c0 + (int64_t)u * kSelThreads;
      if (c < n) f(c, float_key(sgn * v[u] + 0.f));
    }
  }
}

__device__ void select_row_any(SelUnion& u, const float* __restrict__ V, const int32_t* __restrict__ A, int64_t n,
                               int64_t es, int K, bool minimize, float* __restrict__ out_val,
                               int32_t* __restrict__ out_idx, int64_t eo) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (K > n) K = (int)n;
  const float sgn = minimize ? -1.f : 1.f;
  RangeShared& r = u.range.r;
  unsigned long long* keys = u.range.keys;
  // pass 1: key range
  unsigned lo = 0xFFFFFFFFu, hi = 0u;
  for_each_key(V, n, es, sgn, [&](int64_t, unsigned k) {
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  });
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned ol = (unsigned)__shfl_xor((int)lo, off), oh = (unsigned)__shfl_xor((int)hi, off);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  if (lane == 0) {
    r.kmin_w[w] = lo;
    r.kmax_w[w] = hi;
  }
  for (int i = tid; i < kRangeBuckets; i += kSelThreads) r.hist[i] = 0;
  __syncthreads();
  unsigned kmin = r.kmin_w[0], kmax = r.kmax_w[0];
#pragma unroll
  for (int i = 1; i < kSelThreads / 64; ++i) {
    kmin = r.kmin_w[i] < kmin ? r.kmin_w[i] : kmin;
    kmax = r.kmax_w[i] > kmax ? r.kmax_w[i] : kmax;
  }
  const unsigned span = kmax - kmin;
  int shift = 0;
  while ((span >> shift) >= (unsigned)kRangeBuckets) ++shift;
  // pass 2: histogram over the range
  for_each_key(V, n, es, sgn, [&](int64_t, unsigned k) { atomicAdd(&r.hist[(k - kmin) >> shift], 1u); });
  __syncthreads();
  if (tid < 64) {  // one wave: lane l sums buckets [B - PER(l+1), B - PER l), top first
    constexpr int PER = kRangeBuckets / 64;
    unsigned sum = 0;
#pragma unroll 8
    for (int j = 0; j < PER; ++j) sum += r.hist[kRangeBuckets - 1 - PER * lane - j];
    unsigned incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned t = (unsigned)__shfl_up((int)incl, off);
      if (lane >= off) incl += t;
    }
    const unsigned excl = incl - sum;
    if (excl < (unsigned)K && (unsigned)K <= incl) {
      unsigned acc = excl;
      for (int j = 0; j < PER; ++j) {
        const int b = kRangeBuckets - 1 - PER * lane - j;
        const unsigned cnt = r.hist[b];
        if (acc + cnt >= (unsigned)K) {
          r.bstar = b;
          r.above = (int)acc;
          break;
        }
        acc += cnt;
      }
    }
    if (lane == 0) {
      r.nb = 0;
      r.nhi = 0;
    }
  }
  __syncthreads();
  const int bstar = r.bstar, above = r.above;
  if ((int)r.hist[bstar] > kRangeCap) {  // uniform: fall back to the byte-wise select
    __syncthreads();
    select_row(u.radix, V, A, n, es, K, minimize, out_val, out_idx, eo);
    return;
  }
  // pass 3: winners above b*, the b* bucket into LDS
  for_each_key(V, n, es, sgn, [&](int64_t c, unsigned k) {
    const int b = (int)((k - kmin) >> shift);
    if (b >= bstar) {
      const unsigned long long key = ((unsigned long long)k << 32) | unit_lo(A[c * es]);
      if (b > bstar)
        keys[atomicAdd(&r.nhi, 1)] = key;
      else
        r.bnd[atomicAdd(&r.nb, 1)] = key;
    }
  });
  __syncthreads();
  const int nb = r.nb;
  int mb = 1;
  while (mb < nb) mb <<= 1;
  for (int i = nb + tid; i < mb; i += kSelThreads) r.bnd[i] = 0ull;
  __syncthreads();
  bitonic_desc_lds(r.bnd, mb);
  for (int i = tid; i < K - above; i += kSelThreads) keys[above + i] = r.bnd[i];
  int kp = 1;
  while (kp < K) kp <<= 1;
  for (int i = K + tid; i < kp; i += kSelThreads) keys[i] = 0ull;
  __syncthreads();
  bitonic_desc_lds(keys, kp);
  for (int i = tid; i < K; i += kSelThreads) {
    const unsigned long long key = keys[i];
    out_val[i * eo] = sgn * key_float((unsigned)(key >> 32));
    out_idx[i * eo] = unit_code((unsigned)(key & 0xFFFFFFFFull));
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSelThreads) __attribute__((amdgpu_waves_per_eu(8, 10))) void select_kernel(const float* __restrict__ V,
                                                             const int32_t* __restrict__ A, int64_t rows, int64_t n,
                                                             int64_t ldv, int64_t es, int K, int minimize,
                                                             float* __restrict__ out_val,
                                                             int32_t* __restrict__ out_idx, int64_t ldout,
                                                             int64_t eo) {
  __shared__ SelUnion sh;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
    select_row_any(sh, V + r * ldv, A + r * ldv, n, es, K, minimize != 0, out_val + r * ldout,
                   out_idx + r * ldout, eo);
}

__global__ __launch_bounds__(kSelThreads) __attribute__((amdgpu_waves_per_eu(8, 10))) void select_rows_kernel(const SelRow* __restrict__ rows_desc,
                                                                  int64_t rows) {
  __shared__ SelUnion sh;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const SelRow d = rows_desc[r];
    select_row_any(sh, d.V, d.A, d.n, 1, d.K, d.minimize != 0, d.out_val, d.out_idx, 1);
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

// Few results from short rows (K <= 32, n <= 64 R): each lane sorts its R keys, then K
// rounds take the wave's best remaining key (a butterfly maximum over the lanes' heads)
// and the lane holding it drops its head.  About half the instructions of sorting all
// 64 R keys when K is small.  Same order as the other paths.
template <int R>
__global__ __launch_bounds__(256) void select_wave_few_kernel(const float* __restrict__ V,
                                                              const int32_t* __restrict__ A, int64_t rows, int n,
                                                              int64_t ldv, int64_t es, int K, int minimize,
                                                              float* __restrict__ out_val,
                                                              int32_t* __restrict__ out_idx, int64_t ldout,
                                                              int64_t eo) {
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
    // sort the lane's keys, largest first: a bitonic network over the R registers
    // (R log2(R) (log2(R) + 1) / 4 compare-exchanges: 80 for R = 16, where an
    // insertion network takes 120)
#pragma unroll
    for (int size = 2; size <= R; size <<= 1) {
#pragma unroll
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int j = i ^ stride;
          if (j > i) {
            const unsigned long long a = k[i], b = k[j];
            const bool desc = (i & size) == 0;
            const bool sw = desc ? (a < b) : (a > b);
            k[i] = sw ? b : a;
            k[j] = sw ? a : b;
          }
        }
      }
    }
    for (int e = 0; e < K; ++e) {
      unsigned long long m = k[0];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = shfl_xor_u64(m, off);
        m = o > m ? o : m;
      }
      // the lowest lane whose head is the maximum pops it (keys of real candidates are
      // unique; empty slots are all 0 and are never taken before real ones)
      const unsigned long long holders = __ballot(k[0] == m);
      if (lane == __ffsll((long long)holders) - 1) {
#pragma unroll
        for (int i = 0; i + 1 < R; ++i) k[i] = k[i + 1];
        k[R - 1] = 0ull;
      }
      if (lane == 0) {
        out_val[r * ldout + e * eo] = sgn * key_float((unsigned)(m >> 32));
        out_idx[r * ldout + e * eo] = unit_code((unsigned)(m & 0xFFFFFFFFull));
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
  // short rows: a wave per row, sorted in registers; K > 32 over more than 256
  // candidates takes the key-range select instead (the register sort of 512-1024 keys
  // needs 111-209 VGPRs, 2-4 waves per SIMD: FP8 search, L = 704, K_r = 100, 1.52 ->
  // 1.41 ms per step)
  if (n <= 1024 && (K <= 32 || n <= 256)) {
    const int64_t want = ceil_div(rows, 4);
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    const int nn = (int)n, mz = minimize ? 1 : 0;
#define KNN_SELW(R_)                                                                                          \
  do {                                                                                                       \
    if (K <= 32)                                                                                             \
      select_wave_few_kernel<R_><<<grid, 256, 0, s>>>(V, A, rows, nn, ldv, es, K, mz, out_val, out_idx, ldout, \
                                                      eo);                                                   \
    else                                                                                                     \
      select_wave_kernel<R_><<<grid, 256, 0, s>>>(V, A, rows, nn, ldv, es, K, mz, out_val, out_idx, ldout, eo); \
  } while (0)
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
