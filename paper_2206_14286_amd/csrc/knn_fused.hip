// knn_fused.hip -- the distance GEMM fused with the bin-wise partial reduction
// (PartialReduce, Sec. 5, Algorithm 1), for gfx950.
//
// Work item = (query block, bin chunk).  A workgroup of 4 waves owns 4*32*NCB
// queries and a chunk of whole, consecutive bins (rows [r0, r1)), so every bin is
// finished inside one workgroup and the M x N scores never leave the chip
// (the paper's point about aggregating inside the kernel, Sec. 4.2, eq. blas3).
//
//   * Each wave keeps the B operand fragments of its 32*NCB queries in registers
//     for the whole item (the paper's query-block reuse, Algorithm 2's ib loop).
//   * The database streams through LDS in 32-row tiles (Algorithm 2's jb loop):
//     the workgroup copies tiles S ahead with direct buffer->LDS loads while it
//     computes, so each tile is read from L2/HBM once per workgroup.
//   * Scores come from 32x32 MFMA instructions (FP32 32x32x2, BF16 32x32x16,
//     FP8 32x32x64 with a per-row power-of-two scale) with FP32 accumulation.
//     In the 32x32 output layout lane l holds 16 rows of one query column
//     (rows 8*(i/4) + 4*(l/32) + i%4 of the tile, query l%32), so the bin update is
//     per-lane register work.  Algorithm 1 spends a compare and two conditional
//     moves per score; here the running best is updated per group of 4 rows (one
//     max3/max, a compare and two conditional moves per 4 scores), the group's row
//     being found afterwards (knn_resolve.hip), and these instructions are
//     interleaved with the next tile's matrix instructions.
//   * L2 starts the accumulators from -|x|^2/2 (see knn_prepare.hip), so every
//     metric is a maximisation of the accumulator.
//   * A tile with one bin boundary inside updates the bins on either side with
//     masked group updates (exact rows for the one group the boundary splits);
//     tiles at the item's edges or with several boundaries walk their rows in
//     order, exchanging scores between the two lane halves.
//   * Finished bins are staged per wave in LDS and written 16 bins at a time as
//     64-byte row segments.
//   * Bins: contiguous balanced row ranges; ties inside a bin go to the lowest row
//     (strict compare in increasing row order, then lowest unit when the two
//     lane halves are merged).
//   * Workgroup ids are mapped so that the workgroups running on one XCD at a
//     time share the same bin chunk, and its tiles are served from that XCD's L2.
#include <type_traits>

#include "knn_common.cuh"

namespace knn {

namespace {

// Bins leave the kernel through a per-wave LDS window of W consecutive bins x 64
// queries (values and codes), written out as row segments of W bins once the window
// is complete instead of one 4-byte store per query and bin.  Rows of the window
// are padded to W + 1 words (an odd stride) so the per-query writes fall in distinct
// banks.  W = 16 (64-byte segments); 8 for the short FP8 tiles, whose kernel runs four
// waves per SIMD and needs the LDS for a fourth workgroup per CU.
template <int W>
constexpr int stage_words() {
  return 2 * 64 * (W + 1);  // per wave: values, then codes
}

template <int NG>
struct TileGeom {
  static constexpr int kMain = NG * 64;                                     // 16-byte pieces of fragments
  static constexpr int kPerWave = (kMain + 64 * kWaves - 1) / (64 * kWaves);  // fragment loads per wave
  static constexpr int kLoads = kPerWave + 1;                               // + one aux load per wave
  static constexpr int kMainBytes = kPerWave * 64 * kWaves * 16;            // incl. landing pad
  static constexpr int kLdsBytes = kMainBytes + kAuxBytes;
};

// Depths at which the kernel keeps one accumulator set (BF16 from depth 128 up,
// FP8 at depths 128 and 256; see run_item): fewer registers, so two or three waves
// per SIMD overlap one another's bin updates instead of one wave overlapping its
// own.  FP32 keeps the double-buffered form: its matrix instructions are long
// enough that one wave per SIMD keeps the unit busy.
template <int DT, int NG>
constexpr bool kSingleAcc() {
  return (DT == DT_BF16 && NG >= 8) || (DT == DT_FP8 && NG % 4 == 0);
}

// LDS ring depth: 2 for the single-accumulator form (each step refills the buffer
// freed by the previous one; three workgroups per CU fit), 4 for the small-bin FP8
// instance (two tiles per step), 4 for the short double-buffered tiles, 2 for
// FP32-size tiles
template <int DT, int NG, bool kS = false>
constexpr int stages() {
  return kSingleAcc<DT, NG>() ? (kS ? 4 : 2) : (NG <= 8 ? 4 : 2);
}

// kS: the depth-128 FP8 instance for bins of at most 128 rows, whose windows drain
// every few tiles: 16-bin windows (64-byte row segments: fewer partly written lines
// left open in L2 between drains) at three waves per SIMD instead of 8-bin windows at
// four (measured with 64-row bins: 5.6% faster; with bins of thousands of rows 7% slower)
template <int DT, int NG, bool kS = false>
constexpr int win_bins() {
  return (DT == DT_FP8 && NG == 4 && !kS) ? 8 : 16;
}

// Depth split (kSplit, at most 64 queries: one column block for each of two waves):
// waves 0-1 and 2-3 take the two halves of each tile's depth for the same queries, so
// all four SIMDs of a CU do matrix work; the second pair hands its partial sums to the
// first through two LDS buffers of 2 x 64 lanes x 16 floats.
constexpr int kXchgBytes = 2 * 2 * 64 * 16 * 4;

// (output windows for the waves that hold bins: all four, or the first pair when split)
template <int DT, int NG, bool kS = false, bool kSplit = false>
constexpr int lds_bytes() {
  return stages<DT, NG, kS>() * TileGeom<NG>::kLdsBytes +
         (kSplit ? 2 : kWaves) * stage_words<win_bins<DT, NG, kS>()>() * 4 + (kSplit ? kXchgBytes : 0);
}

// wait until at most N vector-memory loads of this wave are outstanding
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Word 3 of a raw buffer descriptor on gfx9-family parts: 32-bit data format, no
// swizzle, no index stride (byte-addressed raw loads).
constexpr int kBufferWord3 = 0x00020000;

// Workgroup barrier without the memory fence __syncthreads() implies.  The fence
// would make the compiler wait for every outstanding direct-to-LDS tile load at
// each barrier, draining the copy pipeline; instead each wave waits explicitly for
// its own loads of the tile about to be read (wait_vmcnt) before the barrier, and
// the asm's memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Per-lane byte offsets of the 16-byte pieces a lane moves when a tile is copied
// into LDS; the same for every tile of an item, so they are computed once and the
// loads use a uniform tile base plus these offsets.
template <int NG>
struct TileLoadPlan {
  unsigned frag_off[TileGeom<NG>::kPerWave];
  unsigned aux_off;
};

// LDS copy of a tile: the global piece layout (knn_internal.h: each group of 4 rows
// contiguous) with the 64-byte sub-blocks of row group rg permuted by XOR with
// (rg % 4) * 64.  Each 16-lane quarter of a copy instruction then reads one aligned
// 256-byte global chunk, and each quarter of a fragment read (16 rows of one
// half, 4 row groups) hits four different 64-byte bank ranges.
template <int NG>
__device__ __forceinline__ int lds_swizzle(int off) {
  return off ^ (((off / (NG * 128)) & 3) << 6);  // an involution: also maps LDS -> global
}

template <int NG>
__device__ __forceinline__ TileLoadPlan<NG> make_load_plan(int wave, int lane) {
  using G = TileGeom<NG>;
  TileLoadPlan<NG> p;
#pragma unroll
  for (int it = 0; it < G::kPerWave; ++it) {
    int k = it * 64 * kWaves + wave * 64 + lane;  // 16-byte LDS slot written by this lane
    k = k < G::kMain ? k : G::kMain - 1;          // pad slots re-read the last piece
    p.frag_off[it] = (unsigned)lds_swizzle<NG>(k * 16);
  }
  p.aux_off = (unsigned)(NG * 1024 + (wave * 4 + (lane & 3)) * 16);
  return p;
}

// copy one prepared tile (NG KiB of fragments + 256 B aux) into LDS with direct
// buffer->LDS loads.  Every wave issues the same number of loads (kLoads): pieces
// past the end re-read the last fragment piece and land in the buffer's pad, and
// each wave moves a quarter of the aux block with four lanes, so per-wave vmcnt
// counts are uniform and a tile's arrival can be awaited with one immediate.
// `wave` must be wave-uniform (an SGPR value): the LDS destination of each load is.
// The buffer form (rather than the flat-encoded global form) matters: the compiler
// counts a flat-encoded LDS load as a possibly out-of-order LDS event and then
// waits for all LDS reads at the first use of any, while after buffer loads it
// waits per fragment.  The descriptor covers exactly the tile (bounds-checked).
template <int NG>
__device__ __forceinline__ void load_tile(const unsigned char* __restrict__ src, unsigned char* lds_dst,
                                          const TileLoadPlan<NG>& p, int wave, int lane) {
  using G = TileGeom<NG>;
  const auto rsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(src), 0, (int)tile_bytes(NG), kBufferWord3);
#pragma unroll
  for (int it = 0; it < G::kPerWave; ++it) {
    unsigned char* dst = lds_dst + (it * 64 * kWaves + wave * 64) * 16;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)(dst), 16, (int)p.frag_off[it],
                                             0, 0, 0);
  }
  if (lane < 4) {
    unsigned char* dst = lds_dst + G::kMainBytes + wave * 64;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)(dst), 16, (int)p.aux_off, 0,
                                             0, 0);
  }
}

// one tile's A operand fragments, accumulator start values (-|x|^2/2 for L2) and
// FP8 row scale, as read from LDS
template <int NG>
struct TileRegs {
  u32x4 af[NG];
  f32x16 init;
  int sa;
};

// kZ: the accumulators start from zero (MIPS, cosine): the start values are not read
// and the first matrix instruction takes an inline zero.  Groups [G0, G0 + NGP) only.
template <int NG, bool kZ, int G0 = 0, int NGP = NG>
__device__ __forceinline__ void read_tile(TileRegs<NG>& r, const unsigned char* tile) {
  using G = TileGeom<NG>;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const float* auxf = reinterpret_cast<const float*>(tile + G::kMainBytes);
  if constexpr (kZ) {
    r.init = f32x16{};
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) r.init[i] = auxf[h * 16 + i];
  }
  r.sa = tile[G::kMainBytes + 128 + (lane & 31)];
  // piece (row q, group g, half h) of the swizzled copy: the XOR flips bit 6 (half)
  // and bit 7 (group parity) of the offset inside the row group's block
  const int q = lane & 31, rg = q >> 2, sw = (rg & 3) << 6;
  const int base = rg * NG * 128 + (q & 3) * 16 + ((h << 6) ^ (sw & 64));
  const int a_even = base + (sw & 128), a_odd = base - (sw & 128);  // (g ^ b7) * 128 = g * 128 +- b7 * 128
#pragma unroll
  for (int g = G0; g < G0 + NGP; ++g)
    r.af[g] = *reinterpret_cast<const u32x4*>(tile + ((g & 1) ? a_odd : a_even) + g * 128);
}

// acc[cb] = init + sum over the tile depth of A(tile rows) x B(query columns)
template <int DT, int NG, int NCB>
__device__ __forceinline__ void mma_tile(f32x16 (&acc)[NCB], const TileRegs<NG>& r, const u32x4 (&bq)[NCB][NG],
                                         const int (&sb)[NCB]) {
  if constexpr (DT == DT_FP8) {
#pragma unroll
    for (int s = 0; s < NG / 2; ++s) {
      const u32x4& a0 = r.af[2 * s];
      const u32x4& a1 = r.af[2 * s + 1];
      i32x8 A = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const u32x4& b0 = bq[cb][2 * s];
        const u32x4& b1 = bq[cb][2 * s + 1];
        i32x8 B = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
        acc[cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, s == 0 ? r.init : acc[cb], 0, 0, 0, r.sa, 0,
                                                                   sb[cb]);
      }
    }
  } else if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      bf16x8 A = __builtin_bit_cast(bf16x8, r.af[g]);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        bf16x8 B = __builtin_bit_cast(bf16x8, bq[cb][g]);
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, g == 0 ? r.init : acc[cb], 0, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(r.af[g][e]), __uint_as_float(bq[cb][g][e]),
                                                         (g == 0 && e == 0) ? r.init : acc[cb], 0, 0, 0);
        }
      }
    }
  }
}

// The matrix instructions of one tile, in fixed order (one k-step for every column
// block, then the next k-step), with the U = 4*NCB units of the previous tile's
// bin update spread evenly between them, two at a time.  A full scheduling barrier after each
// group pins the order: every unit's VALU instructions issue while the matrix
// unit is busy with the group just issued, and alternating column blocks keeps
// consecutive matrix instructions independent.
// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).  Used where
// the body indexes register arrays, so that no trip-count heuristic can leave a
// loop rolled and move the arrays to scratch memory.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Groups [G0, G0 + NGP) of the depth only (the depth-split form).
template <int DT, int NG, int NCB, int G0 = 0, int NGP = NG, class UnitFn>
__device__ __forceinline__ void mma_tile_interleaved(f32x16 (&acc)[NCB], const TileRegs<NG>& r,
                                                     const u32x4 (&bq)[NCB][NG], const int (&sb)[NCB],
                                                     UnitFn&& unit) {
  static_assert(G0 % 2 == 0 && NGP % 2 == 0 && G0 + NGP <= NG, "group range");
  constexpr int P = DT == DT_FP8 ? NGP / 2 : (DT == DT_BF16 ? NGP : 4 * NGP);  // k-steps per column block
  constexpr int U = 4 * NCB;
  static_for<0, P>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    static_for<0, NCB>([&](auto cc) {
      constexpr int cb = decltype(cc)::value;
      if constexpr (DT == DT_FP8) {
        const u32x4& a0 = r.af[G0 + 2 * s];
        const u32x4& a1 = r.af[G0 + 2 * s + 1];
        const u32x4& b0 = bq[cb][G0 + 2 * s];
        const u32x4& b1 = bq[cb][G0 + 2 * s + 1];
        i32x8 A = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
        i32x8 B = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
        acc[cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, s == 0 ? r.init : acc[cb], 0, 0, 0, r.sa, 0,
                                                                   sb[cb]);
      } else if constexpr (DT == DT_BF16) {
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, r.af[G0 + s]),
                                                          __builtin_bit_cast(bf16x8, bq[cb][G0 + s]),
                                                          s == 0 ? r.init : acc[cb], 0, 0, 0);
      } else {
        constexpr int g = G0 + (s >> 2), e = s & 3;
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(r.af[g][e]), __uint_as_float(bq[cb][g][e]),
                                                       s == 0 ? r.init : acc[cb], 0, 0, 0);
      }
    });
    // units go in pairs, so the two independent updates interleave (no stall between
    // a compare and the select that reads its lane mask)
    static_for<0, U / 2>([&](auto pc) {
      constexpr int pr = decltype(pc)::value;
      if constexpr (pr * P / (U / 2) == s) unit(pc);
    });
    __builtin_amdgcn_sched_barrier(0);
  });
}

// acc[cb] = init + the tile's products, with the A fragments read from LDS in chunks
// of 4 groups, each chunk's reads issued before the previous chunk's matrix
// instructions (2 x 4 fragment registers instead of NG).
template <int DT, int NG, int NCB, bool kZ>
__device__ __forceinline__ void mma_tile_chunked(f32x16 (&acc)[NCB], const unsigned char* tile,
                                                 const u32x4 (&bq)[NCB][NG], const int (&sb)[NCB]) {
  using G = TileGeom<NG>;
  constexpr int CH = 4;
  static_assert(NG % CH == 0 && DT != DT_F32, "chunked form: BF16 / FP8, NG a multiple of 4");
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const float* auxf = reinterpret_cast<const float*>(tile + G::kMainBytes);
  f32x16 init = {};
  if constexpr (!kZ) {
#pragma unroll
    for (int i = 0; i < 16; ++i) init[i] = auxf[h * 16 + i];
  }
  const int sa = tile[G::kMainBytes + 128 + (lane & 31)];
  const int q = lane & 31, rg = q >> 2, sw = (rg & 3) << 6;
  const int base = rg * NG * 128 + (q & 3) * 16 + ((h << 6) ^ (sw & 64));
  const int a_even = base + (sw & 128), a_odd = base - (sw & 128);
  u32x4 fa[2][CH];
  auto read_chunk = [&](u32x4 (&f)[CH], int c) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int g = c * CH + j;
      f[j] = *reinterpret_cast<const u32x4*>(tile + ((g & 1) ? a_odd : a_even) + g * 128);
    }
  };
  read_chunk(fa[0], 0);
  static_for<0, NG / CH>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if constexpr (c + 1 < NG / CH) read_chunk(fa[(c + 1) & 1], c + 1);
    if constexpr (DT == DT_BF16) {
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int g = c * CH + j;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[c & 1][j]),
                                                            __builtin_bit_cast(bf16x8, bq[cb][g]),
                                                            g == 0 ? init : acc[cb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int j = 0; j < CH; j += 2) {
        const int g = c * CH + j;
        const u32x4& a0 = fa[c & 1][j];
        const u32x4& a1 = fa[c & 1][j + 1];
        i32x8 A = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const u32x4& b0 = bq[cb][g];
          const u32x4& b1 = bq[cb][g + 1];
          i32x8 B = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
          acc[cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, g == 0 ? init : acc[cb], 0, 0, 0, sa, 0,
                                                                     sb[cb]);
        }
      }
    }
  });
}

// A bin's running winner is a "unit" whose exact row is resolved later from the
// prepared rows (knn_resolve.hip), keyed by its first row s (unsigned, 0xFFFFFFFF = none):
//   row    u = 2 s          one exact row
//   group  u = 2 s + 1      rows s .. s+3 (one lane's accumulators 4k..4k+3)
//   pair   u = 2 s + 3      rows s .. s+3 and s+8 .. s+11 (a lane's accumulators
//                           8p..8p+7: two groups, interleaved with the other half's)
//   quad   u = 2 s + 5      rows s .. s+15 (s a multiple of 16): both halves' pairs
//                           of one 16-row block, when their best scores tie exactly
// Units of one bin never share a row, and two units can interleave only as the two
// halves' pairs of one block (a tie there becomes the quad), so ordering by u orders
// by lowest row.  Inside a lane, group and pair units are kept without the lane
// half's row offset (4 rows for half 1: the same for all of the lane's units), so the
// per-tile update can take them from a scalar; merging the halves adds it back.
constexpr unsigned kNoUnit = 0xFFFFFFFFu;

// a tie between the halves' pairs of one block becomes that block's quad
__device__ __forceinline__ unsigned tie_unit(float v0, unsigned u0, float v1, unsigned u1, unsigned take_u) {
  const bool quad = (v0 == v1) & ((u0 & 7u) == 3u) & ((u1 & 7u) == 3u) & ((u0 >> 5) == (u1 >> 5));
  return quad ? ((u0 & ~31u) | 5u) : take_u;
}

// max(best, a0..a3) folded left to right, which the compiler turns into two v_max3_f32:
// max3(max3(best, a0, a1), a2, a3).  (Nested the other way, it computes the group's
// own maximum first and spends a third instruction on the running best.)  Plain code
// rather than asm, so that the compiler also inserts the wait states that reading a
// matrix instruction's fresh result needs.
__device__ __forceinline__ float max5f(float best, float a0, float a1, float a2, float a3) {
  return fmaxf(fmaxf(fmaxf(fmaxf(best, a0), a1), a2), a3);
}

// Exchanges between the two 32-lane halves of a wave with one VALU swap
// (v_permlane32_swap, no LDS round trip): for x held by every lane, r[0] holds the
// lower half's values in both halves and r[1] the upper half's.
__device__ __forceinline__ unsigned other_half(unsigned x, int h) {  // x of lane l ^ 32
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return h ? r[0] : r[1];
}
__device__ __forceinline__ float other_half(float x, int h) {
  return __uint_as_float(other_half(__float_as_uint(x), h));
}
__device__ __forceinline__ unsigned lower_half(unsigned x) {  // x of lane l & 31
  return __builtin_amdgcn_permlane32_swap(x, x, false, false)[0];
}
__device__ __forceinline__ unsigned upper_half(unsigned x) {  // x of lane 32 + (l & 31)
  return __builtin_amdgcn_permlane32_swap(x, x, false, false)[1];
}

// (value ov, unit ou) beats (v, u): larger value, then lower unit; no short-circuit, so
// it compiles to straight-line selects
__device__ __forceinline__ bool beats(float ov, unsigned ou, float v, unsigned u) {
  return (ov > v) | ((ov == v) & (ou < u));
}

// merge the two lane halves' (value, unit) of one query: larger value, then lower unit
__device__ __forceinline__ void merge_halves(float v, unsigned u, int h, float& mv, unsigned& mu) {
  if (u != kNoUnit && (u & 1u)) u += 8u * (unsigned)h;  // group unit: true first row
  const float ov = other_half(v, h);
  const unsigned ou = other_half(u, h);
  const bool take = beats(ov, ou, v, u);
  mv = take ? ov : v;
  mu = tie_unit(ov, ou, v, u, take ? ou : u);
}

// bins output: value in the metric's sign; a row r >= 0; -2 - s/4 for a group,
// -2 - 2^29 - s/4 for a pair, -2 - 2^30 - s/16 for a quad starting at row s; -1 when
// the bin saw no finite score.  Every form computed, then selected: as a chain of early
// returns it compiles to divergent branches at every bin flush.
__device__ __forceinline__ int32_t bin_code(unsigned u) {
  const int32_t row = (int32_t)(u >> 1), s3 = (int32_t)(u >> 3);
  const int32_t group = -2 - s3, pair = -2 - (1 << 29) - s3, quad = -2 - (1 << 30) - (int32_t)(u >> 5);
  const unsigned t = u & 7u;
  const int32_t odd = t == 1u ? group : (t == 3u ? pair : quad);
  const int32_t c = (u & 1u) ? odd : row;
  return u == kNoUnit ? -1 : c;
}

// put one query's finished bin into the wave's output window
template <int W>
__device__ __forceinline__ void stage_bin(float* st, int qlocal, int bin, float v, unsigned u, float sign) {
  st[qlocal * (W + 1) + (bin & (W - 1))] = sign * v;
  reinterpret_cast<int32_t*>(st)[64 * (W + 1) + qlocal * (W + 1) + (bin & (W - 1))] = bin_code(u);
}

// Write the window of bins [wb, wb + W) clipped to the item's bins [b0, b1) for the
// wave's queries.  Lane (query row ql, part) writes bins wb + 4 part .. + 3 of its row,
// so each store instruction covers W * 4-byte segments of 256 / W rows: as one 16-byte
// store when the row offsets allow it (vec = 4), as two 8-byte stores (vec = 2) or four
// 4-byte ones (vec = 1); bins outside the item are skipped one by one.
template <int NCB, int W>
__device__ __forceinline__ void drain_window(const float* st, int wb, int b0, int b1, float* __restrict__ outV,
                                             int32_t* __restrict__ outA, int64_t ldo, int64_t wq0, int64_t M,
                                             int vec, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  constexpr int P = W / 4, RPI = 64 / P;  // parts per row, rows per instruction
  const int32_t* sa = reinterpret_cast<const int32_t*>(st) + 64 * (W + 1);
#pragma unroll
  for (int s = 0; s < NCB * 32 / RPI; ++s) {
    const int ql = RPI * s + lane / P, part = lane % P;
    const int64_t q = wq0 + ql;
    const int pb = wb + 4 * part;
    const float* sv = st + ql * (W + 1) + 4 * part;
    const int32_t* si = sa + ql * (W + 1) + 4 * part;
    if (q < M) {
      float* ov = outV + q * ldo + pb;
      int32_t* oa = outA + q * ldo + pb;
      if (pb >= b0 && pb + 4 <= b1 && vec == 4) {
        *reinterpret_cast<float4*>(ov) = make_float4(sv[0], sv[1], sv[2], sv[3]);
        *reinterpret_cast<int4*>(oa) = make_int4(si[0], si[1], si[2], si[3]);
      } else if (pb >= b0 && pb + 4 <= b1 && vec == 2) {
        *reinterpret_cast<float2*>(ov) = make_float2(sv[0], sv[1]);
        *reinterpret_cast<float2*>(ov + 2) = make_float2(sv[2], sv[3]);
        *reinterpret_cast<int2*>(oa) = make_int2(si[0], si[1]);
        *reinterpret_cast<int2*>(oa + 2) = make_int2(si[2], si[3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (pb + e >= b0 && pb + e < b1) {
            ov[e] = sv[e];
            oa[e] = si[e];
          }
        }
      }
    }
  }
  // the window's slots are rewritten by the next bins only after these reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Walks the first rows floor(b N / L) of consecutive bins without dividing:
// `next` is the first row of the bin after the current one, rem = (b+1) N mod L.
// next32 is `next` clamped to 2^31 - 1, for the per-tile compares against rows
// t0 + 32 <= N + 31 < 2^31 (32-bit scalar compares instead of 64-bit vector ones).
struct BinCursor {
  int64_t next;
  int next32;
  unsigned rem, nr, L;  // rem, N mod L, L (all < 2^31)
  int64_t nq;           // N / L
  __device__ __forceinline__ int64_t peek2() const { return next + nq + (rem + nr >= L ? 1 : 0); }
  __device__ __forceinline__ void advance() {
    const unsigned r = rem + nr;
    const bool c = r >= L;
    next += nq + (c ? 1 : 0);
    next32 = next < 0x7FFFFFFF ? (int)next : 0x7FFFFFFF;
    rem = c ? r - L : r;
  }
};

__device__ __forceinline__ BinCursor make_cursor(int64_t b, int64_t N, int64_t L) {
  BinCursor c;
  c.next = bin_start(b + 1, N, L);
  c.next32 = c.next < 0x7FFFFFFF ? (int)c.next : 0x7FFFFFFF;
  c.rem = (unsigned)(((b + 1) * N) % L);
  c.nr = (unsigned)(N % L);
  c.L = (unsigned)L;
  c.nq = N / L;
  return c;
}

// kPrio: raise the wave priority while a wave issues a tile's matrix instructions
// (pays off with three waves per SIMD, costs with two).  kSplit: the depth-split form
// (see kXchgBytes): a query block of 64 queries.
template <int DT, int NG, int NCB, bool kPrio, bool kZ, bool kS, bool kSplit = false>
__device__ __forceinline__ void run_item(const unsigned char* __restrict__ db_tiles,
                                         const unsigned char* __restrict__ q_tiles, int64_t N, int64_t L, int64_t M,
                                         int64_t q0, int64_t b0, int64_t b1, float sign, float* __restrict__ outV,
                                         int32_t* __restrict__ outA, int64_t ldo, unsigned char* lds) {
  using G = TileGeom<NG>;
  constexpr int S = stages<DT, NG, kS>();
  static_assert((S & (S - 1)) == 0 && S >= 2, "stages: a power of two >= 2");
  constexpr int64_t TB = (int64_t)NG * 1024 + kAuxBytes;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int h = lane >> 5, ql = lane & 31;
  static_assert(!kSplit || (NCB == 1 && !kSingleAcc<DT, NG>() && NG % 4 == 0), "depth split: one column block");
  // depth split: waves 2-3 compute depth groups [NG/2, NG) for the queries of waves 0-1
  const int part = kSplit ? (wave >> 1) : 0, qwave = kSplit ? (wave & 1) : wave;
  constexpr int NGP = kSplit ? NG / 2 : NG;
  constexpr int W = win_bins<DT, NG, kS>();
  // output window of the wave (split: only the first pair holds bins)
  float* stage = reinterpret_cast<float*>(lds + S * G::kLdsBytes) + qwave * stage_words<W>();
  // the exchange buffer of tile t: float4 i of lane l at [(t & 1) * 2 + qwave][i][l]
  float4* const xchg =
      reinterpret_cast<float4*>(lds + S * G::kLdsBytes + (kSplit ? 2 : kWaves) * stage_words<W>() * 4) +
      qwave * 4 * 64 + lane;
  // widest store the output rows allow (window starts are multiples of 4 bins)
  const uintptr_t oaddr = reinterpret_cast<uintptr_t>(outV) | reinterpret_cast<uintptr_t>(outA);
  const int vec_ok = ((oaddr & 15) == 0 && (ldo & 3) == 0) ? 4 : (((oaddr & 7) == 0 && (ldo & 1) == 0) ? 2 : 1);
  const TileLoadPlan<NG> plan = make_load_plan<NG>(wave, lane);

  // rows and tiles fit in 32 bits (N < 2^31)
  const int r0 = (int)bin_start(b0, N, L), r1 = (int)bin_start(b1, N, L);
  const int t_first = r0 >> 5, t_last = (r1 - 1) >> 5;
  auto buf = [&](int t) { return lds + ((t - t_first) & (S - 1)) * G::kLdsBytes; };

  // query fragments of this wave (tiles of 32 queries; the buffer is padded)
  const int64_t wq0 = q0 + (int64_t)qwave * 32 * NCB;
  u32x4 bq[NCB][NG];
  int sb[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const unsigned char* qt = q_tiles + ((wq0 >> 5) + cb) * TB;
#pragma unroll
    for (int g = 0; g < NG; ++g) bq[cb][g] = *reinterpret_cast<const u32x4*>(qt + piece_offset(ql, g, h, NG));
    sb[cb] = qt[NG * 1024 + 128 + ql];
  }
  const bool active = wq0 < M;

  // running bin state per column block and lane half: best value bv and its unit bu
  float bv[NCB];
  unsigned bu[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    bv[cb] = -INFINITY;
    bu[cb] = kNoUnit;
  }
  int cur_bin = (int)b0;
  BinCursor cursor = make_cursor(b0, N, L);

  // Bin update of one tile, two units at a time: unit u = accumulator group
  // k = u / NCB (rows t0 + 8k + 4h + 0..3) of column block cb = u % NCB, against the
  // running best (groups in row order).
  auto unit_pair = [&](auto pc, f32x16 (&acc_c)[NCB], float (&nbv)[NCB], unsigned (&nbu)[NCB], unsigned gu0) {
      constexpr int pr = decltype(pc)::value;
      constexpr int uA = 2 * pr, uB = 2 * pr + 1;
      constexpr int kA = uA / NCB, cA = uA % NCB, kB = uB / NCB, cB = uB % NCB;
      // two max3 fold a group into the running best; it changed iff the group won
      const f32x16& xA = acc_c[cA];
      const f32x16& xB = acc_c[cB];
      if constexpr (cA != cB) {  // two column blocks: independent states
        const float nA = max5f(nbv[cA], xA[4 * kA], xA[4 * kA + 1], xA[4 * kA + 2], xA[4 * kA + 3]);
        const float nB = max5f(nbv[cB], xB[4 * kB], xB[4 * kB + 1], xB[4 * kB + 2], xB[4 * kB + 3]);
        const bool wA = nA > nbv[cA], wB = nB > nbv[cB];
        nbu[cA] = wA ? gu0 + 16u * kA : nbu[cA];
        nbu[cB] = wB ? gu0 + 16u * kB : nbu[cB];
        nbv[cA] = nA;
        nbv[cB] = nB;
      } else {  // one column block: groups kA < kB update the same state in order
        const float nA = max5f(nbv[cA], xA[4 * kA], xA[4 * kA + 1], xA[4 * kA + 2], xA[4 * kA + 3]);
        const float nB = max5f(nA, xB[4 * kB], xB[4 * kB + 1], xB[4 * kB + 2], xB[4 * kB + 3]);
        const bool wA = nA > nbv[cA], wB = nB > nA;
        nbu[cA] = wA ? gu0 + 16u * kA : nbu[cA];
        nbu[cA] = wB ? gu0 + 16u * kB : nbu[cA];
        nbv[cA] = nB;
      }
  };

  auto flush_all = [&]() {  // the current bin is complete: stage it, open the next
    if constexpr (NCB == 2) {
      // lane half h stages column block h: it keeps its own half's state of block h
      // and receives the other half's, in exchange for its state of block 1 - h
      // (one exchange instead of one per block)
      float kv = h ? bv[1] : bv[0], sv = h ? bv[0] : bv[1];
      unsigned ku = h ? bu[1] : bu[0], su = h ? bu[0] : bu[1];
      const unsigned off = 8u * (unsigned)h;  // group units: the half's first row
      ku += (ku != kNoUnit && (ku & 1u)) ? off : 0u;
      su += (su != kNoUnit && (su & 1u)) ? off : 0u;
      const float ov = other_half(sv, h);
      const unsigned ou = other_half(su, h);
      const bool take = beats(ov, ou, kv, ku);
      stage_bin<W>(stage, h * 32 + ql, cur_bin, take ? ov : kv, tie_unit(ov, ou, kv, ku, take ? ou : ku), sign);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        bv[cb] = -INFINITY;
        bu[cb] = kNoUnit;
      }
    } else {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        float mv;
        unsigned mu;
        merge_halves(bv[cb], bu[cb], h, mv, mu);
        if (h == (cb & 1)) stage_bin<W>(stage, cb * 32 + ql, cur_bin, mv, mu, sign);
        bv[cb] = -INFINITY;
        bu[cb] = kNoUnit;
      }
    }
    if ((cur_bin & (W - 1)) == W - 1 || cur_bin == b1 - 1)
      drain_window<NCB, W>(stage, cur_bin & ~(W - 1), (int)b0, (int)b1, outV, outA, ldo, wq0, M, vec_ok, lane);
    ++cur_bin;
    cursor.advance();
  };

  // Everything after a tile's scores are folded into (nbv, nbu): the fast path,
  // the one-boundary masked path and the row walk, bin flushes.  may_fast false: the
  // caller has already taken the fast case (nbv, nbu are then not used or computed).
  auto finish = [&](auto may_fast, int t0, f32x16 (&acc_c)[NCB], float (&nbv)[NCB], unsigned (&nbu)[NCB]) {
    constexpr bool kMayBeFast = decltype(may_fast)::value;
    const unsigned gu0 = 2u * (unsigned)t0 + 1u;
    // materialise the update here, inside the region with the MFMAs, rather than
    // letting the compiler sink it into the (rarely not taken) fast branch below
    if constexpr (kMayBeFast) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) asm volatile("" : "+v"(nbv[cb]), "+v"(nbu[cb]));
    }
    const int lo = t0 > r0 ? t0 : r0;
    const int hi = (t0 + 32) < r1 ? (t0 + 32) : r1;
    const bool whole = lo == t0 && hi == t0 + 32;  // the tile lies inside the item's rows
    const bool fast = kMayBeFast && whole && t0 + 32 <= cursor.next32;  // whole tile in the current bin
    float obv[NCB];
    unsigned obu[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {  // keep the old state for the row-wise path
      obv[cb] = bv[cb];
      obu[cb] = bu[cb];
      bv[cb] = fast ? nbv[cb] : bv[cb];
      bu[cb] = fast ? nbu[cb] : bu[cb];
    }
    if (fast) {
      if (t0 + 32 == cursor.next32) flush_all();  // the bin ends with this tile
      return;
    }
    if (whole && cursor.peek2() >= t0 + 32) {
      // One bin boundary inside the tile, at row p (the bins on either side hold at
      // least the rest of the tile).  Groups of 4 rows that lie on one side update that
      // side's bin as group units (masked, in straight-line code: branching per group
      // costs registers that the persistent kernel, which holds every depth's code,
      // does not have); only the group containing p (k* = p/8, when p is not a
      // multiple of 4) is split, and it is folded in row by row with exact rows.
      const int p = cursor.next32 - t0;  // 1..31, uniform
      const int kstar = (p & 3) ? (p >> 3) : -1;
      const unsigned gbase = 2u * (unsigned)t0 + 8u * (unsigned)h;  // 2 * (first row of group 0)
      const int h4 = 4 * h;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        float cv = obv[cb], nv = -INFINITY;
        unsigned cu = obu[cb], nu = kNoUnit;
        static_for<0, 4>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          // the lane's group k holds tile rows 8k + 4h + j; row < p  <=>  4h < p - 8k - j
          // (the right side is uniform: a compare against a scalar)
          if (k == kstar) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float a = acc_c[cb][4 * k + j];
              const bool in_cur = h4 < p - 8 * k - j;
              const unsigned code = gbase + 16u * k + 2u * j;
              const float ac = in_cur ? a : -INFINITY, an = in_cur ? -INFINITY : a;
              const bool c1 = ac > cv, c2 = an > nv;
              cv = c1 ? ac : cv;
              cu = c1 ? code : cu;
              nv = c2 ? an : nv;
              nu = c2 ? code : nu;
            }
          } else {
            const float g = fmaxf(fmaxf(fmaxf(acc_c[cb][4 * k], acc_c[cb][4 * k + 1]), acc_c[cb][4 * k + 2]),
                                  acc_c[cb][4 * k + 3]);
            const bool in_cur = h4 < p - 8 * k;  // the whole group is on one side
            const unsigned code = gu0 + 16u * k;  // lane-local group unit
            const float gc = in_cur ? g : -INFINITY, gn = in_cur ? -INFINITY : g;
            const bool c1 = gc > cv, c2 = gn > nv;
            cv = c1 ? gc : cv;
            cu = c1 ? code : cu;
            nv = c2 ? gn : nv;
            nu = c2 ? code : nu;
          }
        });
        bv[cb] = cv;
        bu[cb] = cu;
        obv[cb] = nv;
        obu[cb] = nu;
      }
      flush_all();
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        bv[cb] = obv[cb];
        bu[cb] = obu[cb];
      }
      if (t0 + 32 == cursor.next32) flush_all();  // the next bin ends with the tile too
      return;
    }
    // The tile crosses the item's edge or holds several bin boundaries: walk its rows
    // in order.  Lane (h, ql) follows query ql of column block h (block 0 when NCB is
    // 1); a row's score is read from the lane half that holds it, with one exchange
    // between the halves per row.
    static_assert(NCB <= 2, "the row walk pairs at most two column blocks");
    constexpr int cB = NCB - 1;
    float sv;
    unsigned su;
    {
      float mv;
      unsigned mu;
      merge_halves(obv[0], obu[0], h, mv, mu);
      sv = mv;
      su = mu;
      if (NCB == 2) {
        merge_halves(obv[cB], obu[cB], h, mv, mu);
        if (h == 1) {
          sv = mv;
          su = mu;
        }
      }
    }
    const bool lane_on = h == 0 || NCB == 2;
    auto flush_row = [&]() {
      if (lane_on) stage_bin<W>(stage, h * 32 + ql, cur_bin, sv, su, sign);
      if ((cur_bin & (W - 1)) == W - 1 || cur_bin == b1 - 1)
        drain_window<NCB, W>(stage, cur_bin & ~(W - 1), (int)b0, (int)b1, outV, outA, ldo, wq0, M, vec_ok, lane);
      sv = -INFINITY;
      su = kNoUnit;
      ++cur_bin;
      cursor.advance();
    };
    for (int jj = lo - t0; jj < hi - t0; ++jj) {  // uniform bounds
      const int j = t0 + jj;
      if (j == cursor.next32) flush_row();
      const int ir = 4 * (jj >> 3) + (jj & 3), hr = (jj >> 2) & 1;  // accumulator and lane half of row jj
      const float a = acc_c[0][ir], b = acc_c[cB][ir];
      const float other = other_half(h == 0 ? b : a, h);
      const float x = hr == h ? (h == 0 ? a : b) : other;
      if (x > sv) {
        sv = x;
        su = 2u * (unsigned)j;
      }
    }
    if (hi == cursor.next32) flush_row();
    // back to the per-half form: half 0 carries the open bin's state
    {
      const float vA = __uint_as_float(lower_half(__float_as_uint(sv)));
      const unsigned uA = lower_half(su);
      bv[0] = h == 0 ? vA : -INFINITY;
      bu[0] = h == 0 ? uA : kNoUnit;
      if (NCB == 2) {
        const float vB = __uint_as_float(upper_half(__float_as_uint(sv)));
        const unsigned uB = upper_half(su);
        bv[cB] = h == 0 ? vB : -INFINITY;
        bu[cB] = h == 0 ? uB : kNoUnit;
      }
    }
  };

  if constexpr (kSingleAcc<DT, NG>()) {
    // Large depth: one accumulator set (the double-buffered form needs more than the
    // 256 VGPRs of two waves per SIMD).  Step t: wait for tile t, refill the buffer
    // of tile t-1 with tile t+S-1, then the tile's matrix instructions (fragments
    // read in chunks behind them) and its bin update; the other wave of the SIMD
    // runs its matrix instructions meanwhile.
    f32x16 acc[NCB];
    // one tile: its matrix instructions and its bin update
    auto tile_step = [&](int t) {
      const int t0 = t << 5;
      const unsigned gu0 = 2u * (unsigned)t0 + 1u;
      // a wave issuing its matrix instructions goes first, so the SIMD's other waves
      // fill the gaps with their bin updates instead of delaying the matrix unit
      if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
      mma_tile_chunked<DT, NG, NCB, kZ>(acc, buf(t), bq, sb);
      if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
      // a tile inside the item and inside the current bin (the common case, a uniform
      // test) folds its scores into the running state in place
      if (t0 >= r0 && t0 + 32 <= r1 && t0 + 32 <= cursor.next32) {
        // fold the tile in as pair units: 8 scores per lane per unit, four 3-input
        // maxima, a compare and a select (a quarter fewer instructions than groups)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
          for (int pp = 0; pp < 2; ++pp) {
            const f32x16& a = acc[cb];
            const float n = fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(bv[cb], a[8 * pp]), a[8 * pp + 1]),
                                                                a[8 * pp + 2]), a[8 * pp + 3]), a[8 * pp + 4]),
                                              a[8 * pp + 5]), a[8 * pp + 6]), a[8 * pp + 7]);
            bu[cb] = n > bv[cb] ? gu0 + 2u + 32u * pp : bu[cb];  // pair at row t0 + 16 pp (+ 4 h)
            bv[cb] = n;
          }
        }
        if (t0 + 32 == cursor.next32) flush_all();  // the bin ends with this tile
        return;
      }
      // a tile at an item edge or a bin boundary: the masked path or the row walk
      finish(std::false_type{}, t0, acc, bv, bu);
    };
    if constexpr (kS) {
      // Small bins: two tiles per step and one barrier per step (a ring of 4: the
      // step's two tiles, and the next two loading into the buffers the previous step
      // read).  The flush of a bin every second tile then meets half as many barriers
      // (64-row FP8 bins: 1.72 -> 1.54 ms; with long bins this loop is 1.5% slower).
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
        if (t_first + s2 <= t_last) load_tile<NG>(db_tiles + (int64_t)(t_first + s2) * TB, buf(t_first + s2), plan, wave, lane);
      for (int tp = t_first; tp <= t_last; tp += 2) {
        wait_vmcnt<0>();  // the step's two tiles are the only loads issued before this point
        lds_barrier();
#pragma unroll
        for (int s2 = 2; s2 < 4; ++s2)
          if (tp + s2 <= t_last) load_tile<NG>(db_tiles + (int64_t)(tp + s2) * TB, buf(tp + s2), plan, wave, lane);
        if (!active) continue;
        tile_step(tp);
        if (tp + 1 <= t_last) tile_step(tp + 1);
      }
    } else {
#pragma unroll
      for (int s2 = 0; s2 < S - 1; ++s2)
        if (t_first + s2 <= t_last) load_tile<NG>(db_tiles + (int64_t)(t_first + s2) * TB, lds + s2 * G::kLdsBytes, plan, wave, lane);
      // the next tile to load, advanced by one tile per step (no per-step multiply)
      const unsigned char* src = db_tiles + (int64_t)(t_first + S - 1) * TB;
      for (int t = t_first; t <= t_last; ++t, src += TB) {
        // tiles issued so far: up to min(t + S - 2, t_last); tile t has landed once the
        // later ones are the only loads pending
        if (t_last - t >= S - 2) wait_vmcnt<(S - 2) * G::kLoads>(); else wait_vmcnt<0>();
        lds_barrier();
        if (t + S - 1 <= t_last) load_tile<NG>(src, buf(t + S - 1), plan, wave, lane);
        if (!active) continue;
        tile_step(t);
      }
    }
  } else {
    // Software pipeline over the chunk's tiles.  Step t: the tile loads run S tiles
    // ahead (direct global->LDS); the fragments of tile t+1 are read from LDS and
    // its matrix instructions issued while tile t's scores are folded into the bins,
    // in one scheduling region.  Past the end the pipeline computes on stale LDS
    // data whose results are never used.
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (t_first + s <= t_last) load_tile<NG>(db_tiles + (int64_t)(t_first + s) * TB, lds + s * G::kLdsBytes, plan, wave, lane);
    TileRegs<NG> fr;
    f32x16 acc_a[NCB], acc_b[NCB];
    // depth split: the second wave pair's sums of tile t, handed over through LDS (the
    // step's barrier orders the write before the read; a buffer is rewritten two steps on)
    auto put_partial = [&](const f32x16& a, int t) {
      float4* x = xchg + (t & 1) * 2 * 4 * 64;
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i * 64] = make_float4(a[4 * i], a[4 * i + 1], a[4 * i + 2], a[4 * i + 3]);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // written before the next barrier
    };
    auto add_partial = [&](f32x16& a, int t) {
      const float4* x = xchg + (t & 1) * 2 * 4 * 64;
      float4 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = x[i * 64];
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // read before the next barrier
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[4 * i] += v[i].x;
        a[4 * i + 1] += v[i].y;
        a[4 * i + 2] += v[i].z;
        a[4 * i + 3] += v[i].w;
      }
    };
    auto no_units = [](auto) {};
    if (t_last - t_first >= S - 1) wait_vmcnt<(S - 1) * G::kLoads>(); else wait_vmcnt<0>();
    lds_barrier();
    if (active) {
      if constexpr (kSplit) {
        if (part == 0) {
          read_tile<NG, kZ, 0, NGP>(fr, buf(t_first));
          mma_tile_interleaved<DT, NG, NCB, 0, NGP>(acc_a, fr, bq, sb, no_units);
        } else {
          read_tile<NG, true, NGP, NGP>(fr, buf(t_first));
          mma_tile_interleaved<DT, NG, NCB, NGP, NGP>(acc_a, fr, bq, sb, no_units);
          put_partial(acc_a[0], t_first);
        }
      } else {
        read_tile<NG, kZ>(fr, buf(t_first));
        mma_tile<DT, NG, NCB>(acc_a, fr, bq, sb);
      }
    }
    auto step = [&](int t, f32x16 (&acc_c)[NCB], f32x16 (&acc_n)[NCB]) {
      if (t + 1 <= t_last) {
        // tile t+1 has landed once at most min(S-2, t_last-t-1) later tiles are pending
        if (t_last - t - 1 >= S - 2) wait_vmcnt<(S - 2) * G::kLoads>(); else wait_vmcnt<0>();
      }
      lds_barrier();
      // tile t's fragments were read in the previous step: its buffer takes tile t+S
      if (t + S <= t_last) load_tile<NG>(db_tiles + (int64_t)(t + S) * TB, buf(t), plan, wave, lane);
      if (!active) return;
      if constexpr (kSplit) {
        if (part == 1) {  // the second half of tile t+1's depth, handed to waves 0-1
          read_tile<NG, true, NGP, NGP>(fr, buf(t + 1));
          mma_tile_interleaved<DT, NG, NCB, NGP, NGP>(acc_n, fr, bq, sb, no_units);
          put_partial(acc_n[0], t + 1);
          return;
        }
        add_partial(acc_c[0], t);
      }
      const int t0 = t << 5;
      const unsigned gu0 = 2u * (unsigned)t0 + 1u;  // lane-local unit of accumulator group 0 (uniform)
      float nbv[NCB];
      unsigned nbu[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        nbv[cb] = bv[cb];
        nbu[cb] = bu[cb];
      }
      read_tile<NG, kZ, 0, NGP>(fr, buf(t + 1));
      __builtin_amdgcn_sched_barrier(0);
      mma_tile_interleaved<DT, NG, NCB, 0, NGP>(acc_n, fr, bq, sb, [&](auto pc) { unit_pair(pc, acc_c, nbv, nbu, gu0); });
      finish(std::true_type{}, t0, acc_c, nbv, nbu);
    };
    for (int t = t_first; t <= t_last; t += 2) {
      step(t, acc_a, acc_b);
      if (t + 1 > t_last) break;
      step(t + 1, acc_b, acc_a);
    }
  }
}

// Occupancy: the short FP8 tiles have the least matrix work per tile to hide the bin
// update behind: the depth-128 FP8 kernel runs 4 waves per SIMD (<= 128 VGPRs; its
// output windows of 8 bins leave the LDS for four workgroups per CU), depth 64 FP8
// and the BF16 depth-128 kernel 3 (<= 168 VGPRs).
template <int DT, int NG, bool kS = false>
constexpr int min_waves() {
  return (DT == DT_FP8 && NG == 4) ? (kS ? 3 : 4) : (((DT == DT_FP8 && NG < 4) || (DT == DT_BF16 && NG == 8)) ? 3 : 1);
}

template <int DT, int NG, int NCB, bool kZ, bool kS, bool kSplit = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<DT, NG, kS>(), 8)))
void fused_kernel(FusedParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int64_t chunk = (int64_t)(slot / p.n_qb) * 8 + xcd;
  const int qb = slot % p.n_qb;
  if (chunk >= p.n_chunks) return;
  const int64_t b0 = chunk * p.bins_per_chunk;
  const int64_t b1 = (b0 + p.bins_per_chunk) < p.L ? (b0 + p.bins_per_chunk) : p.L;
  constexpr int64_t QB = (kSplit ? 2 : kWaves) * 32 * NCB;  // queries per block
  run_item<DT, NG, NCB, (min_waves<DT, NG, kS>() >= 3), kZ, kS, kSplit>(p.db_tiles, p.q_tiles, p.N, p.L, p.M, (int64_t)qb * QB,
                                                                         b0, b1, p.out_sign, p.binV, p.binA, p.ldo, lds);
}

template <int DT, int NG, int NCB, bool kZ, bool kS, bool kSplit = false>
hipError_t launch_one(const FusedParams& p, hipStream_t s) {
  (void)hipGetLastError();  // clear any stale error so the check below sees this launch only
  const int64_t per_xcd = ceil_div(p.n_chunks, 8);
  const int64_t grid = 8 * per_xcd * p.n_qb;
  constexpr int lb = lds_bytes<DT, NG, kS, kSplit>();
  {
    const hipError_t e =
        ensure_dynamic_lds(reinterpret_cast<const void*>(&fused_kernel<DT, NG, NCB, kZ, kS, kSplit>), lb);
    if (e != hipSuccess) return e;
  }
  fused_kernel<DT, NG, NCB, kZ, kS, kSplit><<<dim3((unsigned)grid), dim3(64 * kWaves), lb, s>>>(p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- persistent batched form
// the 8 per-XCD item counters start from zero at every launch
__global__ __launch_bounds__(64) void reset_claims_kernel(unsigned* __restrict__ claim) {
  if (threadIdx.x < 8) claim[threadIdx.x] = 0u;
}

template <int DT, int NG, int NCB, bool kZ>
__device__ __forceinline__ void run_group_item(const GroupDesc& gd, const WorkItem& it, unsigned char* lds) {
  run_item<DT, NG, NCB, false, kZ, false>(gd.db_tiles, gd.q_tiles, gd.N, gd.L, gd.M, (int64_t)it.qb * (kWaves * 32 * NCB), it.b0,
                        it.b1, gd.out_sign, gd.binV, gd.binA, gd.ldo, lds);
}

// Held to 2 waves per SIMD (<= 256 VGPRs): with every depth's case inlined the
// compiler would otherwise size the registers for all of them at once.  Items are
// claimed in list order per XCD (a counter bumped by one lane per workgroup), so the
// workgroups running at any moment on an XCD hold neighbouring items, i.e. the query
// blocks of one chunk, and share its tiles in L2 (striding through the list by the
// grid size lets them drift apart).
template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void fused_persistent_kernel(
    const GroupDesc* __restrict__ groups, const WorkItem* __restrict__ items, int64_t n_items,
    unsigned* __restrict__ claim) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ unsigned next_item;
  const int xcd = blockIdx.x & 7;
  const int64_t per_xcd = n_items / 8;
  const WorkItem* list = items + xcd * per_xcd;
  for (;;) {
    __syncthreads();  // the previous item's LDS use and every read of next_item are over
    if (threadIdx.x == 0) next_item = atomicAdd(&claim[xcd], 1u);
    __syncthreads();
    const int64_t k = next_item;
    if (k >= per_xcd) break;  // uniform
    const WorkItem it = list[k];
    if (it.grp < 0) continue;  // padding slot of the per-XCD work lists
    const GroupDesc gd = groups[it.grp];
    switch (gd.ng * 4 + gd.ncb) {
      // BF16 depths 64, 96, 128, 256 (NG = 4, 6, 8, 16) and FP32 / FP8 equivalents
      case 4 * 4 + 1:
        if (gd.zero_init) run_group_item<DT, 4, 1, true>(gd, it, lds); else run_group_item<DT, 4, 1, false>(gd, it, lds);
        break;
      case 4 * 4 + 2:
        if (gd.zero_init) run_group_item<DT, 4, 2, true>(gd, it, lds); else run_group_item<DT, 4, 2, false>(gd, it, lds);
        break;
      case 6 * 4 + 1:
        if (gd.zero_init) run_group_item<DT, 6, 1, true>(gd, it, lds); else run_group_item<DT, 6, 1, false>(gd, it, lds);
        break;
      case 6 * 4 + 2:
        if (gd.zero_init) run_group_item<DT, 6, 2, true>(gd, it, lds); else run_group_item<DT, 6, 2, false>(gd, it, lds);
        break;
      case 8 * 4 + 1:
        if (gd.zero_init) run_group_item<DT, 8, 1, true>(gd, it, lds); else run_group_item<DT, 8, 1, false>(gd, it, lds);
        break;
      case 8 * 4 + 2:
        if (gd.zero_init) run_group_item<DT, 8, 2, true>(gd, it, lds); else run_group_item<DT, 8, 2, false>(gd, it, lds);
        break;
      case 16 * 4 + 1:
        if (gd.zero_init) run_group_item<DT, 16, 1, true>(gd, it, lds); else run_group_item<DT, 16, 1, false>(gd, it, lds);
        break;
      case 16 * 4 + 2:
        if (gd.zero_init) run_group_item<DT, 16, 2, true>(gd, it, lds); else run_group_item<DT, 16, 2, false>(gd, it, lds);
        break;
      default: break;
    }
  }
}

}  // namespace

int fused_lds_bytes(int dt, int ng, int ncb) {
  (void)ncb;
#define KNN_LDS_CASE(D_)                 \
  if (dt == D_) switch (ng) {            \
      case 2: return lds_bytes<D_, 2>();   \
      case 4: return lds_bytes<D_, 4>();   \
      case 6: return lds_bytes<D_, 6>();   \
      case 8: return lds_bytes<D_, 8>();   \
      case 12: return lds_bytes<D_, 12>(); \
      case 16: return lds_bytes<D_, 16>(); \
      case 24: return lds_bytes<D_, 24>(); \
      default: return lds_bytes<D_, 32>(); \
    }
  KNN_LDS_CASE(DT_F32)
  KNN_LDS_CASE(DT_BF16)
  KNN_LDS_CASE(DT_FP8)
#undef KNN_LDS_CASE
  return lds_bytes<DT_F32, 32>();
}

#define KNN_FUSED_CASES(X)                                                                                     \
  X(DT_F32, 4, 1) X(DT_F32, 4, 2) X(DT_F32, 8, 1) X(DT_F32, 8, 2) X(DT_F32, 12, 1) X(DT_F32, 12, 2)            \
  X(DT_F32, 16, 1) X(DT_F32, 16, 2) X(DT_F32, 24, 1) X(DT_F32, 32, 1)                                          \
  X(DT_BF16, 2, 1) X(DT_BF16, 2, 2) X(DT_BF16, 4, 1) X(DT_BF16, 4, 2) X(DT_BF16, 6, 1) X(DT_BF16, 6, 2)        \
  X(DT_BF16, 8, 1) X(DT_BF16, 8, 2) X(DT_BF16, 12, 1) X(DT_BF16, 12, 2) X(DT_BF16, 16, 1) X(DT_BF16, 16, 2)    \
  X(DT_FP8, 2, 1) X(DT_FP8, 2, 2) X(DT_FP8, 4, 1) X(DT_FP8, 4, 2) X(DT_FP8, 6, 1) X(DT_FP8, 6, 2)              \
  X(DT_FP8, 8, 1) X(DT_FP8, 8, 2)

bool fused_supported(int dt, int ng, int ncb) {
#define X(D_, G_, C_) \
  if (dt == D_ && ng == G_ && ncb == C_) return true;
  KNN_FUSED_CASES(X)
#undef X
  return false;
}

hipError_t launch_fused(int dt, int ng, int ncb, const FusedParams& p, hipStream_t s) {
  if (p.M == 0 || p.n_chunks == 0) return hipSuccess;
  if (dt == DT_F32 && ncb == 1 && p.M <= 64) {  // one query block of at most 64 queries: depth split
#define X(G_)        \
  if (ng == G_)      \
    return p.zero_init ? launch_one<DT_F32, G_, 1, true, false, true>(p, s) : launch_one<DT_F32, G_, 1, false, false, true>(p, s);
    X(4) X(8) X(12) X(16) X(24) X(32)
#undef X
  }
  if (dt == DT_FP8 && ng == 4 && p.N <= 128 * p.L) {  // bins of at most 128 rows
    if (ncb == 2)
      return p.zero_init ? launch_one<DT_FP8, 4, 2, true, true>(p, s) : launch_one<DT_FP8, 4, 2, false, true>(p, s);
    if (ncb == 1)
      return p.zero_init ? launch_one<DT_FP8, 4, 1, true, true>(p, s) : launch_one<DT_FP8, 4, 1, false, true>(p, s);
  }
#define X(D_, G_, C_) \
  if (dt == D_ && ng == G_ && ncb == C_) \
    return p.zero_init ? launch_one<D_, G_, C_, true, false>(p, s) : launch_one<D_, G_, C_, false, false>(p, s);
  KNN_FUSED_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fused_persistent(int dt, const GroupDesc* d_groups, const WorkItem* d_items, int64_t n_items,
                                   unsigned* d_claim, int n_blocks, int lds_bytes_needed, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  if (dt != DT_BF16) return hipErrorInvalidValue;  // the batched form is built for BF16 databases
  if (n_items % 8 != 0 || n_items / 8 >= (int64_t(1) << 31) || n_blocks % 8 != 0) return hipErrorInvalidValue;
  const int lb = lds_bytes_needed;
  (void)hipGetLastError();
  {
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&fused_persistent_kernel<DT_BF16>), lb);
    if (e != hipSuccess) return e;
  }
  reset_claims_kernel<<<1, 64, 0, s>>>(d_claim);
  fused_persistent_kernel<DT_BF16><<<n_blocks, 64 * kWaves, lb, s>>>(d_groups, d_items, n_items, d_claim);
  return hipGetLastError();
}

}  // namespace knn
