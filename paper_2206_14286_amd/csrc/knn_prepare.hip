// knn_prepare.hip -- row preparation for the distance kernel.
//
// One thread per row; a workgroup's 64 rows are first staged in LDS with coalesced
// loads (the batched query segments read their rows directly).  For cosine the row is
// unit-normalised in FP32 (|x|^2
// summed in dimension order with one rounding per product and per sum, correctly
// rounded square root and divisions), which makes cosine search an inner-product
// search (Sec. 2: MIPS equals cosine search on l2-normalised data).  The row is
// then converted to the compute type, zero-padded to the MFMA depth (the paper
// pads GloVe's D = 100 to 128, appendix "Benchmark details") and scattered into
// the piece layout described in knn_internal.h.  For L2 the aux block gets
// -|x~|^2/2 of the converted row: the distance kernel starts its accumulators
// from it, so <q,x> - |x|^2/2 (the negated relaxed distance of eq. l2final)
// comes out of the matrix unit with no extra per-score instruction.
#include "knn_common.cuh"

namespace knn {

namespace {

// Element d of a row in FP32 (0 past D or for a padding row), from global memory or
// from a copy staged in LDS.
struct GlobalRow {
  const void* src;
  int dt;
  int64_t base;
  __device__ __forceinline__ float operator()(int d) const { return load_elem(src, dt, base + d); }
};
struct LdsRow {
  const float* row;
  __device__ __forceinline__ float operator()(int d) const { return row[d]; }
};

// source row r (valid if r < rows) -> destination row dst of `tiles`
template <int CDT, class Src>
__device__ void prepare_row(const Src& load, bool valid, int64_t r, int64_t dst, int D, int ng, int metric,
                            bool database, unsigned char* tiles, float* orig_half_norm, float* orig_rnorm) {
  // one rounding per product and per sum: no fused multiply-add in this function
#pragma clang fp contract(off)
  float ss = 0.f;
  if (valid)
    for (int d0 = 0; d0 < D; d0 += 16) {  // 16 loads in flight, summed in dimension order
      float x[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = d0 + k < D ? load(d0 + k) : 0.f;
#pragma unroll
      for (int k = 0; k < 16; ++k) ss = ss + x[k] * x[k];
    }
  const float nrm = sqrtf(ss);  // correctly rounded square root (HIP default)
  if (valid && orig_half_norm) orig_half_norm[r] = 0.5f * ss;
  if (valid && orig_rnorm) orig_rnorm[r] = nrm > 0.f ? 1.f / nrm : 0.f;
  const bool cosine = metric == MET_COSINE;
  auto get = [&](int d) -> float {
    if (!valid || d >= D) return 0.f;
    const float x = load(d);
    if (!cosine) return x;
    return nrm > 0.f ? x / nrm : 0.f;  // correctly rounded division (HIP default)
  };

  int e = 0;
  if (CDT == DT_FP8) {
    float amax = 0.f;
    for (int d0 = 0; d0 < D; d0 += 16) {
      float x[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = get(d0 + k);
#pragma unroll
      for (int k = 0; k < 16; ++k) amax = fmaxf(amax, fabsf(x[k]));
    }
    e = fp8_row_exponent(amax);
  }
  const float down = exp2i(-e), up = exp2i(e);

  constexpr int E = CDT == DT_F32 ? 4 : (CDT == DT_BF16 ? 8 : 16);  // elements per 16 bytes
  const int64_t tile = dst >> 5;
  const int rr = (int)(dst & 31);
  unsigned char* tb = tiles + tile * tile_bytes(ng);
  float hh = 0.f;
  for (int g = 0; g < ng; ++g) {
    for (int hf = 0; hf < 2; ++hf) {
      const int d0 = g * 2 * E + hf * E;
      u32x4 w = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int k = 0; k < E; ++k) {
        float x = get(d0 + k);
        float deq;
        unsigned bits;
        if (CDT == DT_F32) {
          bits = __float_as_uint(x);
          deq = x;
          w[k] = bits;
        } else if (CDT == DT_BF16) {
          bits = bf16_rne(x);
          deq = __uint_as_float(bits << 16);
          w[k >> 1] |= bits << (16 * (k & 1));
        } else {
          bits = fp8_e4m3_rne(x * down);
          deq = fp8_e4m3_value(bits) * up;
          w[k >> 2] |= bits << (8 * (k & 3));
        }
        hh = hh + deq * deq;
      }
      *reinterpret_cast<u32x4*>(tb + piece_offset(rr, g, hf, ng)) = w;
    }
  }
  unsigned char* aux = tb + ng * 1024;
  const int half = (rr >> 2) & 1, idx = 4 * (rr >> 3) + (rr & 3);
  reinterpret_cast<float*>(aux)[half * 16 + idx] = (database && metric == MET_L2) ? -0.5f * hh : 0.f;
  aux[128 + rr] = (unsigned char)(e + 127);
}

// The 64 rows of a workgroup are consecutive in the source, so they are first copied
// into LDS with coalesced loads (consecutive threads, consecutive elements) by all 256
// threads, 8 loads each in flight (one trip to memory for rows of up to 128 FP32
// elements), widened to FP32 (exact), one row per LDS row of D + 1 words (an odd
// stride: thread t reading element d of its own row hits bank (t (D + 1) + d) mod 64,
// a different bank per thread).  The first 64 threads then prepare one row each from
// LDS with the arithmetic above.
constexpr int kPrepRows = 64;
constexpr int kPrepThreads = 256;

template <int CDT>
__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(const void* src, int in_dt, int64_t rows, int D, int ng,
                                                             int metric, int database, unsigned char* tiles,
                                                             int64_t n_rows_padded, float* orig_half_norm,
                                                             float* orig_rnorm) {
  extern __shared__ float stage[];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kPrepRows;
  const int64_t nrow = src == nullptr ? 0 : (rows - r0 < kPrepRows ? (rows - r0 > 0 ? rows - r0 : 0) : kPrepRows);
  const int total = (int)nrow * D;  // <= 64 * 256
  const int64_t base = r0 * (int64_t)D;
  // row of staged element i: floor((i + 1/2) / D) in FP32 is exact here, since (i + 1/2) / D
  // is at least 1/(2D) away from an integer and i < 2^14
  const float inv_d = 1.f / (float)D;
  auto put = [&](int i, float x) {
    const int rr = (int)(((float)i + 0.5f) * inv_d), d = i - rr * D;
    stage[rr * (D + 1) + d] = x;
  };
  const int esz = in_dt == DT_F32 ? 4 : 2;
  if (reinterpret_cast<uintptr_t>(src) % 16 == 0 && (D * esz) % 16 == 0) {
    // 16-byte loads (the block's rows are one aligned span): 8 per thread in flight
    const int per = 16 / esz, total16 = total / per;
    const u32x4* s16 = reinterpret_cast<const u32x4*>(static_cast<const unsigned char*>(src) + base * esz);
    constexpr int U = 8;
    for (int i0 = 0; i0 < total16; i0 += kPrepThreads * U) {
      u32x4 w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kPrepThreads + t;
        w[u] = i < total16 ? s16[i] : u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kPrepThreads + t;
        if (i >= total16) continue;
        if (in_dt == DT_F32) {
#pragma unroll
          for (int k = 0; k < 4; ++k) put(i * 4 + k, __uint_as_float(w[u][k]));
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const unsigned h = (k & 1) ? (w[u][k >> 1] >> 16) : (w[u][k >> 1] & 0xFFFFu);
            put(i * 8 + k, __uint_as_float(h << 16));
          }
        }
      }
    }
  } else {
    constexpr int U = 8;
    for (int i0 = 0; i0 < total; i0 += kPrepThreads * U) {
      float x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kPrepThreads + t;
        x[u] = i < total ? load_elem(src, in_dt, base + i) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kPrepThreads + t;
        if (i < total) put(i, x[u]);
      }
    }
  }
  __syncthreads();
  const int64_t r = r0 + t;
  if (t >= kPrepRows || r >= n_rows_padded) return;
  prepare_row<CDT>(LdsRow{stage + t * (D + 1)}, src != nullptr && r < rows, r, r, D, ng, metric, database != 0,
                   tiles, orig_half_norm, orig_rnorm);
}

// One wave per row, so that a few rows do not leave one thread per row doing all of
// its work serially.  Lane l holds elements l, l + 64, ... of the row; the sums that
// have an order (|x|^2 for cosine and the original-row norms, the L2 half norm of the
// converted row) are taken by lane 0 in dimension order with one rounding per product
// and per sum, as prepare_row takes them; the FP8 row maximum is a wave reduction (a
// maximum in any order is exact), and lane p < 2 NG converts and stores piece p.
// Produces the same bytes as prepare_row.
constexpr int kWPrepWaves = 4;

template <int CDT>
__global__ __launch_bounds__(64 * kWPrepWaves) void prepare_rows_wave_kernel(
    const void* src, int in_dt, int64_t rows, int D, int ng, int metric, int database, unsigned char* tiles,
    int64_t n_rows_padded, float* orig_half_norm, float* orig_rnorm) {
#pragma clang fp contract(off)
  __shared__ float stage[kWPrepWaves][kMaxDpad];
  __shared__ float dq[kWPrepWaves][kMaxDpad];  // dequantised converted row (L2 database half norm)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * kWPrepWaves + w;
  if (r >= n_rows_padded) return;
  const bool valid = src != nullptr && r < rows;
  float* row = stage[w];
#pragma unroll
  for (int j = 0; j < kMaxDpad / 64; ++j) {
    const int d = 64 * j + lane;
    row[d] = (valid && d < D) ? load_elem(src, in_dt, r * (int64_t)D + d) : 0.f;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const bool cosine = metric == MET_COSINE;
  const bool need_ss = cosine || orig_half_norm != nullptr || orig_rnorm != nullptr;
  float nrm = 0.f;
  if (need_ss) {
    float ss = 0.f;
    if (lane == 0)
      for (int d = 0; d < D; ++d) ss = ss + row[d] * row[d];
    ss = __shfl(ss, 0);
    nrm = sqrtf(ss);  // correctly rounded square root (HIP default)
    if (lane == 0 && valid && orig_half_norm) orig_half_norm[r] = 0.5f * ss;
    if (lane == 0 && valid && orig_rnorm) orig_rnorm[r] = nrm > 0.f ? 1.f / nrm : 0.f;
  }
  auto get = [&](int d) -> float {
    const float x = row[d];  // 0 past D and for padding rows
    if (!cosine) return x;
    return nrm > 0.f ? x / nrm : 0.f;  // correctly rounded division (HIP default)
  };
  int e = 0;
  if (CDT == DT_FP8) {
    float amax = 0.f;
#pragma unroll
    for (int j = 0; j < kMaxDpad / 64; ++j) {
      const int d = 64 * j + lane;
      if (d < D) amax = fmaxf(amax, fabsf(get(d)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    e = fp8_row_exponent(amax);
  }
  const float down = exp2i(-e), up = exp2i(e);
  constexpr int E = CDT == DT_F32 ? 4 : (CDT == DT_BF16 ? 8 : 16);  // elements per 16 bytes
  unsigned char* tb = tiles + (r >> 5) * tile_bytes(ng);
  const int rr = (int)(r & 31);
  const bool half_norm = database != 0 && metric == MET_L2;
  if (lane < 2 * ng) {
    const int g = lane >> 1, hf = lane & 1;
    const int d0 = g * 2 * E + hf * E;
    u32x4 wv = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int d = d0 + k;
      const float x = d < D ? get(d) : 0.f;
      float deq;
      if (CDT == DT_F32) {
        wv[k] = __float_as_uint(x);
        deq = x;
      } else if (CDT == DT_BF16) {
        const unsigned bits = bf16_rne(x);
        wv[k >> 1] |= bits << (16 * (k & 1));
        deq = __uint_as_float(bits << 16);
      } else {
        const unsigned bits = fp8_e4m3_rne(x * down);
        wv[k >> 2] |= bits << (8 * (k & 3));
        deq = fp8_e4m3_value(bits) * up;
      }
      if (half_norm) dq[w][d] = deq;
    }
    *reinterpret_cast<u32x4*>(tb + piece_offset(rr, g, hf, ng)) = wv;
  }
  float hh = 0.f;
  if (half_norm) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0)
      for (int d = 0; d < 2 * ng * E; ++d) hh = hh + dq[w][d] * dq[w][d];
  }
  if (lane == 0) {
    unsigned char* aux = tb + ng * 1024;
    const int half = (rr >> 2) & 1, idx = 4 * (rr >> 3) + (rr & 3);
    reinterpret_cast<float*>(aux)[half * 16 + idx] = half_norm ? -0.5f * hh : 0.f;
    aux[128 + rr] = (unsigned char)(e + 127);
  }
}

template <int CDT>
__global__ __launch_bounds__(64) void prepare_segments_kernel(const QSeg* segs, int nseg, int64_t total_rows,
                                                               int in_dt) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total_rows) return;
  int lo = 0, hi = nseg - 1;  // last segment with first <= r
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= r) lo = mid; else hi = mid - 1;
  }
  const QSeg& s = segs[lo];
  const int64_t local = r - s.first;  // rows past s.rows are padding
  prepare_row<CDT>(GlobalRow{s.src, in_dt, local * (int64_t)s.D}, s.src != nullptr && local < s.rows, local,
                   s.dst_row0 + local, s.D, s.ng, s.metric, false, s.tiles, nullptr, nullptr);
}

}  // namespace

hipError_t launch_prepare(const void* src, int in_dt, int64_t rows, int D, int metric, int compute,
                          bool database, unsigned char* tiles, int64_t n_tiles, float* orig_half_norm,
                          float* orig_rnorm, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  const int ng = groups_for(dpad_for(D, compute), compute);
  const int64_t n = n_tiles * kTileRows;
  if (n == 0) return hipSuccess;
  // One wave per row for queries, and for database rows that need no ordered sum (MIPS
  // without original-row norms): measured 2.74 -> 1.98 ms for 4M x 256 BF16 rows.  Rows
  // whose half norm or cosine norm is summed in order keep one thread per row: lane 0
  // of a wave summing alone is slower there (1M x 128 L2: 0.28 -> 0.74 ms).
  if (!database || (metric == MET_MIPS && !orig_half_norm && !orig_rnorm)) {
    const unsigned wgrid = (unsigned)ceil_div(n, kWPrepWaves);
    const int db = database ? 1 : 0;
    if (compute == DT_F32)
      prepare_rows_wave_kernel<DT_F32><<<wgrid, 64 * kWPrepWaves, 0, s>>>(src, in_dt, rows, D, ng, metric, db, tiles, n,
                                                                         orig_half_norm, orig_rnorm);
    else if (compute == DT_BF16)
      prepare_rows_wave_kernel<DT_BF16><<<wgrid, 64 * kWPrepWaves, 0, s>>>(src, in_dt, rows, D, ng, metric, db, tiles,
                                                                          n, orig_half_norm, orig_rnorm);
    else
      prepare_rows_wave_kernel<DT_FP8><<<wgrid, 64 * kWPrepWaves, 0, s>>>(src, in_dt, rows, D, ng, metric, db, tiles, n,
                                                                         orig_half_norm, orig_rnorm);
    return hipGetLastError();
  }
  const unsigned grid = (unsigned)ceil_div(n, kPrepRows);
  const size_t lds = sizeof(float) * kPrepRows * (size_t)(D + 1);  // <= 65,792 bytes (D <= 256)
  {
    const void* fn = compute == DT_F32    ? reinterpret_cast<const void*>(&prepare_kernel<DT_F32>)
                     : compute == DT_BF16 ? reinterpret_cast<const void*>(&prepare_kernel<DT_BF16>)
                                          : reinterpret_cast<const void*>(&prepare_kernel<DT_FP8>);
    const hipError_t e = ensure_dynamic_lds(fn, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (compute == DT_F32)
    prepare_kernel<DT_F32><<<grid, kPrepThreads, lds, s>>>(src, in_dt, rows, D, ng, metric, database, tiles, n,
                                                        orig_half_norm, orig_rnorm);
  else if (compute == DT_BF16)
    prepare_kernel<DT_BF16><<<grid, kPrepThreads, lds, s>>>(src, in_dt, rows, D, ng, metric, database, tiles, n,
                                                         orig_half_norm, orig_rnorm);
  else
    prepare_kernel<DT_FP8><<<grid, kPrepThreads, lds, s>>>(src, in_dt, rows, D, ng, metric, database, tiles, n,
                                                        orig_half_norm, orig_rnorm);
  return hipGetLastError();
}

hipError_t launch_prepare_segments(const QSeg* d_segs, int nseg, int64_t total_rows, int in_dt, int compute,
                                   hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  if (total_rows == 0 || nseg == 0) return hipSuccess;
  const unsigned grid = (unsigned)ceil_div(total_rows, 64);
  if (compute == DT_F32)
    prepare_segments_kernel<DT_F32><<<grid, 64, 0, s>>>(d_segs, nseg, total_rows, in_dt);
  else if (compute == DT_BF16)
    prepare_segments_kernel<DT_BF16><<<grid, 64, 0, s>>>(d_segs, nseg, total_rows, in_dt);
  else
    prepare_segments_kernel<DT_FP8><<<grid, 64, 0, s>>>(d_segs, nseg, total_rows, in_dt);
  return hipGetLastError();
}

}  // namespace knn
