// knn_approx.hip -- PartialReduce over a score matrix the caller already holds: the
// approx_max_k / approx_min_k op on its own (App. A.1 lists its options; the reduction
// is Sec. 5, Algorithm 1, without the distance GEMM in front of it).
//
// The op reads every score once and does a compare and a select per score, so it is
// bound by HBM bandwidth (the regime of eq. blas3), not by the matrix units.
//
//   approx_rows_kernel: bins along the contiguous dimension (each row of the matrix is
//     one slice).  A workgroup owns a run of whole bins of one row.  Each wave reads a
//     4 KB span per pass with fully coalesced 16-byte loads, passes it through a
//     wave-private LDS buffer so that every lane ends up with 4 consecutive 16-byte
//     pieces (16 FP32 or 32 BF16 consecutive scores), and keeps a running
//     (value, index) winner for the bin its scores are in.  Scores are compared in
//     increasing index order with a strict comparison, so the lowest index wins ties,
//     as in Algorithm 1.  A lane hands its winner to the bin's LDS slot when it leaves
//     the bin, as a 64-bit key
//       float_key(sgn * v + 0) << 32 | ~j   (sgn = -1 for minimisation),
//     merged with an LDS atomic max: the larger key is the better score and, for equal
//     scores, the lower index.  Adding +0 maps -0 to +0 so the two zeros tie.
//   approx_cols_kernel: bins down the strided dimension (each column is one slice).  A
//     lane owns one column and walks its rows in order through a run of bins; a wave
//     reads 64 consecutive columns of one row per load.  Bins of at least 256 rows are
//     split into quarters over the workgroup's four waves, merged in order through LDS.
#include <algorithm>
#include <cmath>

#include "knn_common.cuh"

namespace knn {

namespace {

constexpr int kApproxThreads = 256;
constexpr int kApproxWaves = kApproxThreads / 64;
constexpr int kApproxMaxItemBins = 1024;   // bins one workgroup keeps in LDS
constexpr double kApproxItemCols = 65536;  // target scores per row work item
constexpr int64_t kApproxMinItems = 4096;  // work items wanted when the matrix allows
constexpr double kApproxItemRows = 2048;   // target rows per column work item

__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

template <bool MIN>
__device__ __forceinline__ bool better(float a, float b) {
  return MIN ? (a < b) : (a > b);
}

template <bool MIN>
__device__ __forceinline__ unsigned long long win_key(float v, int32_t j) {
  const float s = MIN ? -v : v;
  return ((unsigned long long)float_key(s + 0.f) << 32) | (unsigned long long)(~(uint32_t)j);
}

template <bool MIN>
__device__ __forceinline__ void write_key(unsigned long long key, float* v, int32_t* a) {
  const float s = key_float((unsigned)(key >> 32));
  *v = MIN ? -s : s;
  *a = (int32_t)(~(uint32_t)(key & 0xFFFFFFFFull));
}

// One 16-byte piece of a row: elements [e, e + VEC) where e < c1 (the item's end).
// Elements at or beyond c1 are not read (they may lie past the allocation).
template <typename T, bool ALIGNED>
__device__ __forceinline__ u32x4 load_piece(const T* row, int64_t e, int64_t c1) {
  constexpr int VEC = 16 / sizeof(T);
  if (e >= c1) return u32x4{0u, 0u, 0u, 0u};
  if (ALIGNED && e + VEC <= c1) return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row + e));
  T v[VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) v[i] = (e + i < c1) ? row[e + i] : T(0);
  u32x4 u;
  __builtin_memcpy(&u, v, 16);
  return u;
}

template <typename T>
__device__ __forceinline__ float piece_elem(const u32x4& u, int i) {
  if constexpr (sizeof(T) == 4) {
    const unsigned w = u[i];
    return __uint_as_float(w);
  } else {
    const unsigned w = u[i >> 1];
    return __uint_as_float((i & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
}

// Bins along rows.  Work item it = (row r, bins [b0, b0 + nb)), nb <= kApproxMaxItemBins,
// covering columns [c0, c1) = [start(b0), start(b0 + nb)).  The item is read in passes of
// kApproxThreads * 4 pieces; the first piece starts at c0 rounded down to a piece
// boundary when rows are 16-byte aligned (ALIGNED), else at c0.
template <typename T, bool ALIGNED, bool MIN>
__global__ __launch_bounds__(kApproxThreads) void approx_rows_kernel(const T* __restrict__ S, int64_t B, int64_t n,
                                                                     int64_t ld, int64_t L, int64_t bpi,
                                                                     int64_t ipr, uint32_t l_mul,
                                                                     float* __restrict__ outV,
                                                                     int32_t* __restrict__ outA) {
  constexpr int VEC = 16 / sizeof(T);  // scores per piece
  constexpr int EPL = 4 * VEC;         // scores per lane per pass
  constexpr int64_t WSPAN = 256 * VEC; // scores per wave per pass
  __shared__ unsigned long long slot[kApproxMaxItemBins];
  __shared__ int32_t start[kApproxMaxItemBins + 1];
  __shared__ u32x4 stage[kApproxWaves][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // Load instruction u of a wave reads pieces 64u .. 64u + 63 of its span (one
  // contiguous KB); lane t takes piece 64u + perm(t) and stores it at LDS slot 64u + t.
  // Lane t then reads slots 64(t/16) + 16v + t%16 (v = 0..3), which hold pieces
  // 4t + v: its 4 consecutive pieces.  Both LDS access patterns are free of bank
  // conflicts (16 consecutive lanes cover all 16 16-byte bank groups).
  const int perm = 4 * (lane & 15) + (lane >> 4);
  const int rd = 64 * (lane >> 4) + (lane & 15);
  const int64_t n_items = B * ipr;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int64_t r = it / ipr;
    const int64_t b0 = (it - r * ipr) * bpi;
    const int nb = (int)(L - b0 < bpi ? L - b0 : bpi);
    for (int i = tid; i <= nb; i += kApproxThreads) start[i] = (int32_t)bin_start(b0 + i, n, L);
    for (int i = tid; i < nb; i += kApproxThreads) slot[i] = 0ull;
    __syncthreads();
    const int64_t c0 = start[0], c1 = start[nb];
    const T* row = S + r * ld;
    const int64_t first = ALIGNED ? (c0 & ~(int64_t)(VEC - 1)) : c0;
    // running winner of this lane: bin cb (relative; -1 none), value bv at index bj
    int cb = -1;
    int32_t next = 0, bj = 0;
    float bv = 0.f;
    // leave the current bin (hand its winner to the slot) and enter the bin of j
    auto enter = [&](int32_t j) {
      if (cb >= 0) atomicMax(&slot[cb], win_key<MIN>(bv, bj));
      // bin of j is floor(((j+1) L - 1) / n); l_mul = floor(2^32 L / n) gives
      // floor((j+1) L / n) or one less (one 32 x 32 -> 64-bit multiply, no division),
      // within 2 of it; the two loops below make it exact
      int64_t be = (int64_t)(((uint64_t)(uint32_t)(j + 1) * l_mul) >> 32) - b0;
      int b = (int)(be < 0 ? 0 : (be >= nb ? nb - 1 : be));
      while (b > 0 && start[b] > j) --b;
      while (start[b + 1] <= j) ++b;
      cb = b;
      next = start[b + 1];
    };
    u32x4 pc[4];
    {
      const int64_t wb = first + w * WSPAN;
#pragma unroll
      for (int u = 0; u < 4; ++u) pc[u] = load_piece<T, ALIGNED>(row, wb + (int64_t)(64 * u + perm) * VEC, c1);
    }
    for (int64_t pbase = first; pbase < c1; pbase += kApproxWaves * WSPAN) {
      const int64_t wb = pbase + w * WSPAN;
#pragma unroll
      for (int u = 0; u < 4; ++u) stage[w][64 * u + lane] = pc[u];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      u32x4 mine[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) mine[v] = stage[w][rd + 16 * v];
      // next pass's pieces are in flight while this pass is reduced
      const int64_t nwb = wb + kApproxWaves * WSPAN;
#pragma unroll
      for (int u = 0; u < 4; ++u) pc[u] = load_piece<T, ALIGNED>(row, nwb + (int64_t)(64 * u + perm) * VEC, c1);
      const int64_t j0l = wb + (int64_t)lane * EPL;  // index of this lane's first score
      const int64_t lo = c0 - j0l > 0 ? c0 - j0l : 0, hi = c1 - j0l < EPL ? c1 - j0l : EPL;
      if (lo < hi) {
        const int32_t j0 = (int32_t)j0l;  // j0 + lo < c1 < 2^31
        bool fresh = false;               // the lane's first valid score opens bin cb
        if (cb < 0 || j0 + (int32_t)lo >= next) {
          enter(j0 + (int32_t)lo);
          fresh = true;
        }
        if (lo == 0 && hi == EPL && j0 + EPL <= next) {
          // All of the lane's scores lie in bin cb.  Their best value m (a max/min tree,
          // two scores per instruction) replaces the running winner only if strictly
          // better, and then at the first position holding m: the same result as
          // comparing the scores one by one in increasing order.
          float x[EPL];
#pragma unroll
          for (int i = 0; i < EPL; ++i) x[i] = piece_elem<T>(mine[i / VEC], i % VEC);
          float m = x[0];
#pragma unroll
          for (int i = 1; i + 1 < EPL; i += 2)
            m = MIN ? fminf(m, fminf(x[i], x[i + 1])) : fmaxf(m, fmaxf(x[i], x[i + 1]));
          if constexpr (EPL % 2 == 0) m = MIN ? fminf(m, x[EPL - 1]) : fmaxf(m, x[EPL - 1]);
          if (fresh || better<MIN>(m, bv)) {
            int idx = EPL - 1;
#pragma unroll
            for (int i = EPL - 2; i >= 0; --i) idx = (x[i] == m) ? i : idx;
            bv = m;
            bj = j0 + idx;
          }
        } else {
          // a bin boundary (or the item's edge) inside the lane's scores: one by one
#pragma unroll
          for (int i = 0; i < EPL; ++i) {
            if (i < lo || i >= hi) continue;
            const float xi = piece_elem<T>(mine[i / VEC], i % VEC);
            const int32_t j = j0 + i;
            if (fresh && i == lo) {
              bv = xi;
              bj = j;
            } else if (j >= next) {
              enter(j);
              bv = xi;
              bj = j;
            } else if (better<MIN>(xi, bv)) {
              bv = xi;
              bj = j;
            }
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (cb >= 0) atomicMax(&slot[cb], win_key<MIN>(bv, bj));
    __syncthreads();
    for (int i = tid; i < nb; i += kApproxThreads) write_key<MIN>(slot[i], outV + r * L + b0 + i, outA + r * L + b0 + i);
    __syncthreads();
  }
}

// Bins down columns.  Work item = (block of 64 columns, bins [b0, b0 + bpi)); lane l of
// every wave owns column c = 64 * block + l, so a wave reads 64 consecutive columns of one
// row per load, UNR rows per step with the loads issued first.  Bin starts advance without
// division: with n = qL + rem, start(b + 1) = start(b) + q + carry.
//   split (bins of many rows): the 4 waves scan consecutive quarters of each bin's rows
//     and the quarters' winners are merged in order through LDS (a strictly better later
//     quarter replaces an earlier one, so the lowest row still wins ties);
//   otherwise wave w takes every 4th bin of the item on its own.
// Output bins are laid out bin-major: V[b * B + c].
template <typename T, bool MIN>
__device__ __forceinline__ void scan_rows(const T* __restrict__ col, int64_t ld, int64_t rs, int64_t re, float& bv,
                                          int64_t& bj) {
  constexpr int UNR = 16;
  bv = widen(col[rs * ld]);
  bj = rs;
  for (int64_t j = rs + 1; j < re; j += UNR) {
    T v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) v[u] = (j + u < re) ? col[(j + u) * ld] : T(0);
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const float x = widen(v[u]);
      if (j + u < re && better<MIN>(x, bv)) {
        bv = x;
        bj = j + u;
      }
    }
  }
}

template <typename T, bool MIN>
__global__ __launch_bounds__(kApproxThreads) void approx_cols_kernel(const T* __restrict__ S, int64_t B, int64_t n,
                                                                     int64_t ld, int64_t L, int64_t bpi,
                                                                     int64_t n_cblk, int split,
                                                                     float* __restrict__ outV,
                                                                     int32_t* __restrict__ outA) {
  __shared__ float part_v[kApproxWaves][64];
  __shared__ int64_t part_j[kApproxWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n_items = n_cblk * ((L + bpi - 1) / bpi);
  const int64_t q = n / L, rem = n - q * L;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int64_t blk = it % n_cblk, bi = it / n_cblk;
    const int64_t c = blk * 64 + lane;
    const bool valid = c < B;
    const T* col = S + (valid ? c : 0);
    const int64_t b0 = bi * bpi, b1 = (b0 + bpi < L) ? b0 + bpi : L;
    int64_t s = bin_start(b0, n, L);
    int64_t frac = (int64_t)(((unsigned long long)b0 * (unsigned long long)rem) % (unsigned long long)L);
    for (int64_t b = b0; b < b1; ++b) {
      frac += rem;
      const int64_t e = s + q + (frac >= L ? 1 : 0);
      if (frac >= L) frac -= L;
      if (split) {
        const int64_t rs = s + ((e - s) * w) / kApproxWaves, re = s + ((e - s) * (w + 1)) / kApproxWaves;
        float bv = 0.f;
        int64_t bj = -1;
        if (valid && rs < re) scan_rows<T, MIN>(col, ld, rs, re, bv, bj);
        part_v[w][lane] = bv;
        part_j[w][lane] = bj;
        __syncthreads();
        if (w == 0 && valid) {
          float v = 0.f;
          int64_t j = -1;
#pragma unroll
          for (int p = 0; p < kApproxWaves; ++p) {
            const int64_t pj = part_j[p][lane];
            if (pj >= 0 && (j < 0 || better<MIN>(part_v[p][lane], v))) {
              v = part_v[p][lane];
              j = pj;
            }
          }
          outV[b * B + c] = v;
          outA[b * B + c] = (int32_t)j;
        }
        __syncthreads();
      } else if ((int)((b - b0) % kApproxWaves) == w && valid) {
        float bv;
        int64_t bj;
        scan_rows<T, MIN>(col, ld, s, e, bv, bj);
        outV[b * B + c] = bv;
        outA[b * B + c] = (int32_t)bj;
      }
      s = e;
    }
  }
}

unsigned grid_for(int64_t items) { return (unsigned)(items < 16384 ? items : 16384); }

template <typename T, bool MIN>
void launch_rows(const T* S, int64_t B, int64_t n, int64_t ld, int64_t L, float* outV, int32_t* outA,
                 hipStream_t s) {
  int64_t bpi = (int64_t)(kApproxItemCols * (double)L / (double)n);
  bpi = bpi < 1 ? 1 : (bpi > kApproxMaxItemBins ? kApproxMaxItemBins : bpi);
  if (bpi > L) bpi = L;
  // smaller items when there are too few to fill the chip, down to one pass of scores
  const int64_t want_ipr = (kApproxMinItems + B - 1) / B;
  if ((L + bpi - 1) / bpi < want_ipr) {
    const int64_t pass_bins = (int64_t)std::ceil((double)kApproxThreads * 64.0 / sizeof(T) * (double)L / (double)n);
    bpi = std::max<int64_t>(std::max<int64_t>(L / want_ipr, pass_bins), 1);
    bpi = std::min<int64_t>(bpi, std::min<int64_t>(L, kApproxMaxItemBins));
  }
  const int64_t ipr = (L + bpi - 1) / bpi;
  const unsigned grid = grid_for(B * ipr);
  // floor(2^32 L / n), saturated at L = n: a fixed-point L / n for the bin estimate
  const uint64_t lm = (uint64_t)(((unsigned __int128)L << 32) / (unsigned __int128)n);
  const uint32_t l_mul = lm > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)lm;
  const bool aligned = (reinterpret_cast<uintptr_t>(S) % 16 == 0) && ((ld * (int64_t)sizeof(T)) % 16 == 0);
  if (aligned)
    approx_rows_kernel<T, true, MIN><<<grid, kApproxThreads, 0, s>>>(S, B, n, ld, L, bpi, ipr, l_mul, outV, outA);
  else
    approx_rows_kernel<T, false, MIN><<<grid, kApproxThreads, 0, s>>>(S, B, n, ld, L, bpi, ipr, l_mul, outV, outA);
}

template <typename T, bool MIN>
void launch_cols(const T* S, int64_t B, int64_t n, int64_t ld, int64_t L, float* outV, int32_t* outA,
                 hipStream_t s) {
  const bool split = (double)n / (double)L >= 256.0;
  const int64_t n_cblk = (B + 63) / 64;
  int64_t bpi = (int64_t)(kApproxItemRows * (double)L / (double)n);
  bpi = bpi < 1 ? 1 : (bpi > L ? L : bpi);
  if (!split) bpi = std::max<int64_t>(bpi, kApproxWaves);  // every wave gets bins
  bpi = std::min<int64_t>(bpi, L);
  const unsigned grid = grid_for(n_cblk * ((L + bpi - 1) / bpi));
  approx_cols_kernel<T, MIN><<<grid, kApproxThreads, 0, s>>>(S, B, n, ld, L, bpi, n_cblk, split ? 1 : 0, outV, outA);
}

template <typename T>
void launch_typed(const void* S, int64_t rows, int64_t cols, int64_t ld, int dim, int64_t L, bool minimize,
                  float* outV, int32_t* outA, hipStream_t s) {
  const T* p = static_cast<const T*>(S);
  if (dim == 1) {
    if (minimize)
      launch_rows<T, true>(p, rows, cols, ld, L, outV, outA, s);
    else
      launch_rows<T, false>(p, rows, cols, ld, L, outV, outA, s);
  } else {
    if (minimize)
      launch_cols<T, true>(p, cols, rows, ld, L, outV, outA, s);
    else
      launch_cols<T, false>(p, cols, rows, ld, L, outV, outA, s);
  }
}

}  // namespace

hipError_t launch_approx_bins(const void* S, int dt, int64_t rows, int64_t cols, int64_t ld, int dim, int64_t L,
                              bool minimize, float* outV, int32_t* outA, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  if ((dim == 1 ? rows : cols) == 0) return hipSuccess;
  if (dt == DT_F32)
    launch_typed<float>(S, rows, cols, ld, dim, L, minimize, outV, outA, s);
  else
    launch_typed<unsigned short>(S, rows, cols, ld, dim, L, minimize, outV, outA, s);
  return hipGetLastError();
}

}  // namespace knn
