// knn_resolve.hip -- exact rows for bin winners recorded as 4-row groups.
//
// The distance kernel tracks, per lane, the best of each group of 4 accumulators
// (4 consecutive database rows) instead of the best single accumulator; that
// halves the per-score instruction count of the bin update.  A winner recorded
// as a group is resolved here: one wave recomputes the group's 4 scores from the
// same prepared (converted) rows and query the matrix unit used, in FP32 with a
// fixed order (16 lanes per row, each a 16-byte piece, then a butterfly), and
// keeps the best row, the lower row on ties.  The result can differ from the
// matrix unit's choice only when two rows of the group score within rounding of
// each other.
#include "knn_common.cuh"

namespace knn {

namespace {

template <int DT>
__device__ __forceinline__ float piece_dot(const u32x4& a, const u32x4& b) {
  float s = 0.f;
  if constexpr (DT == DT_F32) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s = fmaf(__uint_as_float(a[k]), __uint_as_float(b[k]), s);
  } else if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned wa = a[k >> 1] >> (16 * (k & 1)), wb = b[k >> 1] >> (16 * (k & 1));
      s = fmaf(__uint_as_float((wa & 0xFFFFu) << 16), __uint_as_float((wb & 0xFFFFu) << 16), s);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const unsigned ca = (a[k >> 2] >> (8 * (k & 3))) & 0xFFu, cb = (b[k >> 2] >> (8 * (k & 3))) & 0xFFu;
      s = fmaf(fp8_e4m3_value(ca), fp8_e4m3_value(cb), s);
    }
  }
  return s;
}

// resolve one code in place; the calling wave is uniform on (q_tile, qrow, code)
template <int DT>
__device__ __forceinline__ void resolve_one(int32_t* p, const unsigned char* __restrict__ q_tiles, int64_t qrow,
                                            const unsigned char* __restrict__ db_tiles, int ng) {
  const int lane = threadIdx.x & 63;
  const int32_t code = *p;
  if (code > -2) return;
  const int64_t start = (int64_t)(-2 - code) * 4;
  const int r = lane >> 4, pl = lane & 15;
  const int64_t row = start + r;
  const int64_t TB = tile_bytes(ng);
  const unsigned char* dtile = db_tiles + (row >> 5) * TB;
  const unsigned char* qtile = q_tiles + (qrow >> 5) * TB;
  const int rr = (int)(row & 31), qq = (int)(qrow & 31);
  float dot = 0.f;
  for (int pc = pl; pc < 2 * ng; pc += 16) {
    const int g = pc >> 1, hf = pc & 1;
    const u32x4 a = *reinterpret_cast<const u32x4*>(dtile + g * 1024 + (rr + 32 * hf) * 16);
    const u32x4 b = *reinterpret_cast<const u32x4*>(qtile + g * 1024 + (qq + 32 * hf) * 16);
    dot += piece_dot<DT>(a, b);
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) dot += __shfl_xor(dot, off);
  if constexpr (DT == DT_FP8) {
    const int ea = (int)dtile[ng * 1024 + 128 + rr] - 127, eb = (int)qtile[ng * 1024 + 128 + qq] - 127;
    dot = dot * exp2i(ea) * exp2i(eb);
  }
  const float* init = reinterpret_cast<const float*>(dtile + ng * 1024);
  float v = init[((rr >> 2) & 1) * 16 + 4 * (rr >> 3) + (rr & 3)] + dot;
  int best = r;
#pragma unroll
  for (int off = 16; off < 64; off <<= 1) {
    const float ov = __shfl_xor(v, off);
    const int ob = __shfl_xor(best, off);
    const bool take = (ov > v) || (ov == v && ob < best);
    v = take ? ov : v;
    best = take ? ob : best;
  }
  if (lane == 0) *p = (int32_t)(start + best);
}

template <int DT>
__global__ __launch_bounds__(256) void resolve_kernel(int32_t* __restrict__ codes, int64_t rows, int64_t cols,
                                                      int64_t ld, const unsigned char* __restrict__ q_tiles,
                                                      const unsigned char* __restrict__ db_tiles, int ng) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= rows * cols) return;
  const int64_t i = e / cols, c = e % cols;
  resolve_one<DT>(codes + i * ld + c, q_tiles, i, db_tiles, ng);
}

template <int DT>
__global__ __launch_bounds__(256) void resolve_rows_kernel(const SelRow* __restrict__ rows_desc, int64_t rows) {
  const int wave = threadIdx.x >> 6;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const SelRow d = rows_desc[r];
    for (int k = wave; k < d.K; k += 4) resolve_one<DT>(d.out_idx + k, d.q_tiles, d.q_row, d.db_tiles, d.ng);
  }
}

}  // namespace

hipError_t launch_resolve(int dt, int32_t* codes, int64_t rows, int64_t cols, int64_t ld,
                          const unsigned char* q_tiles, const unsigned char* db_tiles, int ng, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)ceil_div(n, 4);
  if (dt == DT_F32)
    resolve_kernel<DT_F32><<<grid, 256, 0, s>>>(codes, rows, cols, ld, q_tiles, db_tiles, ng);
  else if (dt == DT_BF16)
    resolve_kernel<DT_BF16><<<grid, 256, 0, s>>>(codes, rows, cols, ld, q_tiles, db_tiles, ng);
  else
    resolve_kernel<DT_FP8><<<grid, 256, 0, s>>>(codes, rows, cols, ld, q_tiles, db_tiles, ng);
  return hipGetLastError();
}

hipError_t launch_resolve_rows(int dt, const SelRow* d_rows, int64_t rows, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  if (rows == 0) return hipSuccess;
  const unsigned grid = (unsigned)(rows < 65536 ? rows : 65536);
  if (dt == DT_F32)
    resolve_rows_kernel<DT_F32><<<grid, 256, 0, s>>>(d_rows, rows);
  else if (dt == DT_BF16)
    resolve_rows_kernel<DT_BF16><<<grid, 256, 0, s>>>(d_rows, rows);
  else
    resolve_rows_kernel<DT_FP8><<<grid, 256, 0, s>>>(d_rows, rows);
  return hipGetLastError();
}

}  // namespace knn
