// knn_resolve.hip -- exact rows for bin winners recorded as groups of rows.
//
// The distance kernel tracks, per lane, the best of each group of 4 accumulators
// (4 consecutive database rows), or of each pair of such groups, instead of the best
// single accumulator; that cuts the per-score instruction count of the bin update.
// A winner recorded as a group (4 rows), a pair (rows s..s+3 and s+8..s+11) or a
// quad (16 consecutive rows) is resolved here: a group of 16 lanes recomputes the
// scores of each 4-row block, in increasing row order, from the same prepared
// (converted) rows and query the matrix unit used, in FP32 with a fixed order (each
// lane a strided set of 16-byte pieces, then a butterfly across the 16 lanes), and
// keeps the best row, the lower row on ties.  The result can differ from the matrix
// unit's choice only when two rows score within rounding of each other.
#include "knn_common.cuh"

namespace knn {

namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));

// dot product of two 16-byte pieces (4 FP32, 8 BF16 or 16 FP8 elements), FP32 FMAs
// in element order.  FP8-e4m3 codes are widened with the hardware conversion
// (exact: every e4m3 value is an FP32 value).
template <int DT>
__device__ __forceinline__ float piece_dot(const u32x4& a, const u32x4& b, float s) {
  if constexpr (DT == DT_F32) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s = fmaf(__uint_as_float(a[k]), __uint_as_float(b[k]), s);
  } else if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s = fmaf(__uint_as_float(a[k] << 16), __uint_as_float(b[k] << 16), s);
      s = fmaf(__uint_as_float(a[k] & 0xFFFF0000u), __uint_as_float(b[k] & 0xFFFF0000u), s);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const f32x2 a0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)a[k], false), a1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)a[k], true);
      const f32x2 b0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)b[k], false), b1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)b[k], true);
      s = fmaf(a0[0], b0[0], s);
      s = fmaf(a0[1], b0[1], s);
      s = fmaf(a1[0], b1[0], s);
      s = fmaf(a1[1], b1[1], s);
    }
  }
  return s;
}

// Resolve one code in place with a group of 16 lanes (gl = lane within the group,
// all 16 lanes pass the same p).  Lane gl takes pieces gl, gl+16, ... of the four
// rows and of the query row; the four partial sums are reduced across the group
// with a fixed butterfly, so every lane ends with all four scores.  The best row
// wins, the lower row on ties.
template <int DT>
__device__ __forceinline__ void resolve16(int32_t* p, const unsigned char* __restrict__ q_tiles, int64_t qrow,
                                          const unsigned char* __restrict__ db_tiles, int ng, int gl) {
  const int32_t code = *p;
  if (code > -2) return;  // already a row (or no winner)
  // the code's 4-row blocks, in increasing row order: (first row, step between blocks, count)
  int64_t first;
  int step, nblk;
  if (code > -2 - (1 << 29)) {  // group
    first = (int64_t)(-2 - code) * 4;
    step = 0;
    nblk = 1;
  } else if (code > -2 - (1 << 30)) {  // pair
    first = (int64_t)(-2 - (1 << 29) - code) * 4;
    step = 8;
    nblk = 2;
  } else {  // quad
    first = (int64_t)(-2 - (1 << 30) - code) * 16;
    step = 4;
    nblk = 4;
  }
  const int64_t TB = tile_bytes(ng);
  const unsigned char* dtile = db_tiles + (first >> 5) * TB;  // the blocks share the tile
  const unsigned char* qtile = q_tiles + (qrow >> 5) * TB;
  const int qq = (int)(qrow & 31);
  const float* init = reinterpret_cast<const float*>(dtile + ng * 1024);
  if (2 * ng <= 8) {
    // Rows of at most 8 pieces (FP8 depth <= 128, BF16 <= 64, FP32 <= 32): the two 8-lane
    // halves take alternate blocks (half hb: blocks hb, hb + 2), one piece per lane, an
    // 8-lane butterfly (the same sums as the 16-lane one, whose upper lanes would add
    // zeros), then the halves merge by larger value, then lower row: the row a scan in
    // increasing row order with a strict compare keeps.
    const int hb = gl >> 3, g8 = gl & 7;
    float hv = -INFINITY;
    int hbest = -1;  // row within the tile
    for (int blk = hb; blk < nblk; blk += 2) {
      const int r0 = (int)(first & 31) + blk * step;
      float dot[4] = {0.f, 0.f, 0.f, 0.f};
      if (g8 < 2 * ng) {
        const int g = g8 >> 1, hf = g8 & 1;
        const u32x4 b = *reinterpret_cast<const u32x4*>(qtile + piece_offset(qq, g, hf, ng));
        const unsigned char* a = dtile + piece_offset(r0, g, hf, ng);
        u32x4 ar[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) ar[r] = *reinterpret_cast<const u32x4*>(a + r * 16);
#pragma unroll
        for (int r = 0; r < 4; ++r) dot[r] = piece_dot<DT>(ar[r], b, dot[r]);
      }
#pragma unroll
      for (int off = 4; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) dot[r] += __shfl_xor(dot[r], off, 8);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = r0 + r;
        float d = dot[r];
        if constexpr (DT == DT_FP8) {
          const int ea = (int)dtile[ng * 1024 + 128 + rr] - 127, eb = (int)qtile[ng * 1024 + 128 + qq] - 127;
          d = d * exp2i(ea) * exp2i(eb);
        }
        const float v = init[((rr >> 2) & 1) * 16 + 4 * (rr >> 3) + (rr & 3)] + d;
        if (hbest < 0 || v > hv) {
          hv = v;
          hbest = rr;
        }
      }
    }
    const float ov = __shfl_xor(hv, 8, 16);
    const int ob = __shfl_xor(hbest, 8, 16);
    if (ob >= 0 && (hbest < 0 || ov > hv || (ov == hv && ob < hbest))) hbest = ob;
    if (gl == 0) *p = (int32_t)((first & ~(int64_t)31) + hbest);
    return;
  }
  float bv = -INFINITY;
  int64_t best = first;
  for (int blk = 0; blk < nblk; ++blk) {
    const int r0 = (int)(first & 31) + blk * step;
    float dot[4] = {0.f, 0.f, 0.f, 0.f};
    for (int pc = gl; pc < 2 * ng; pc += 16) {
      const int g = pc >> 1, hf = pc & 1;
      const u32x4 b = *reinterpret_cast<const u32x4*>(qtile + piece_offset(qq, g, hf, ng));
      const unsigned char* a = dtile + piece_offset(r0, g, hf, ng);  // the 4 rows' pieces are adjacent
      u32x4 ar[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) ar[r] = *reinterpret_cast<const u32x4*>(a + r * 16);
#pragma unroll
      for (int r = 0; r < 4; ++r) dot[r] = piece_dot<DT>(ar[r], b, dot[r]);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1)
#pragma unroll
      for (int r = 0; r < 4; ++r) dot[r] += __shfl_xor(dot[r], off, 16);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = r0 + r;
      float d = dot[r];
      if constexpr (DT == DT_FP8) {
        const int ea = (int)dtile[ng * 1024 + 128 + rr] - 127, eb = (int)qtile[ng * 1024 + 128 + qq] - 127;
        d = d * exp2i(ea) * exp2i(eb);
      }
      const float v = init[((rr >> 2) & 1) * 16 + 4 * (rr >> 3) + (rr & 3)] + d;
      if ((blk == 0 && r == 0) || v > bv) {  // strict, rows in increasing order: the lower row keeps ties
        bv = v;
        best = (first & ~(int64_t)31) + rr;
      }
    }
  }
  if (gl == 0) *p = (int32_t)best;
}

template <int DT>
__global__ __launch_bounds__(256) void resolve_kernel(int32_t* __restrict__ codes, int64_t rows, int64_t cols,
                                                      int64_t ld, const unsigned char* __restrict__ q_tiles,
                                                      const unsigned char* __restrict__ db_tiles, int ng) {
  const int gl = threadIdx.x & 15;
  const int64_t n = rows * cols;
  const int64_t groups = (int64_t)gridDim.x * 16;
  for (int64_t e = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4); e < n; e += groups) {
    const int64_t i = e / cols, c = e - i * cols;
    resolve16<DT>(codes + i * ld + c, q_tiles, i, db_tiles, ng, gl);
  }
}

template <int DT>
__global__ __launch_bounds__(256) void resolve_rows_kernel(const SelRow* __restrict__ rows_desc, int64_t rows) {
  const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const SelRow d = rows_desc[r];
    for (int k = grp; k < d.K; k += 16) resolve16<DT>(d.out_idx + k, d.q_tiles, d.q_row, d.db_tiles, d.ng, gl);
  }
}

}  // namespace

hipError_t launch_resolve(int dt, int32_t* codes, int64_t rows, int64_t cols, int64_t ld,
                          const unsigned char* q_tiles, const unsigned char* db_tiles, int ng, hipStream_t s) {
  (void)hipGetLastError();  // report only this call's launch errors
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  // 16 codes per workgroup per pass; enough workgroups to fill the chip, then a grid-stride loop
  const int64_t want = ceil_div(n, 16);
  const unsigned grid = (unsigned)(want < 8192 ? want : 8192);
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
