// knn_fused.hip -- the distance GEMM fused with the bin-wise partial reduction
// (PartialReduce, Sec. 4, Algorithm 1), for gfx950.
//
// Work item = (query block, bin chunk).  A workgroup of 4 waves owns 4*32*NCB
// queries and a chunk of whole, consecutive bins (rows [r0, r1)), so every bin is
// finished inside one workgroup and the M x N scores never leave the chip
// (the paper's point about aggregating inside the kernel, Sec. 3.2, eq. blas3).
//
//   * Each wave keeps the B operand fragments of its 32*NCB queries in registers
//     for the whole item (the paper's query-block reuse, Algorithm 2's ib loop).
//   * The database streams through LDS in 32-row tiles (Algorithm 2's jb loop):
//     the whole workgroup copies tile t+1 with direct global->LDS loads while it
//     computes tile t, so each tile is read from L2/HBM once per workgroup.
//   * Scores come from 32x32 MFMA instructions (FP32 32x32x2, BF16 32x32x16,
//     FP8 32x32x64 with a per-row power-of-two scale) with FP32 accumulation.
//     In the 32x32 output layout lane l holds 16 rows of one query column
//     (rows 8*(i/4) + 4*(l/32) + i%4 of the tile, query l%32), so the bin update is
//     per-lane register work: one compare and two conditional moves per score,
//     the 3 COPs of Algorithm 1, against a running (best value, row) pair.
//   * L2 starts the accumulators from -|x|^2/2 (see knn_prepare.hip), so every
//     metric is a maximisation of the accumulator.
//   * Tiles that straddle a bin boundary or the chunk edge take a slower path:
//     the wave spills the tile's scores to its private LDS scratch and one lane
//     per query walks the 32 rows in order, closing bins as it crosses them.
//   * Bins: contiguous balanced row ranges; ties inside a bin go to the lowest row
//     (strict compare in increasing row order, then lowest index when the two
//     lane halves are merged).
//   * Workgroup ids are mapped so that the workgroups running on one XCD at a
//     time share the same bin chunk, and its tiles are served from that XCD's L2.
#include "knn_common.cuh"

namespace knn {

namespace {

constexpr int kSlowFloats = 2 * 32 * 33;  // per-wave scratch: 2 column blocks x 32 queries x 33

template <int NG>
struct TileGeom {
  static constexpr int kChunks = NG * 64 + kAuxBytes / 16;        // 16-byte pieces of a tile
  static constexpr int kPerWave = (kChunks + 64 * kWaves - 1) / (64 * kWaves);
  static constexpr int kLdsBytes = kPerWave * 64 * kWaves * 16;    // buffer incl. landing pad
};

template <int NG, int NCB>
constexpr int lds_bytes() {
  return 2 * TileGeom<NG>::kLdsBytes + kWaves * kSlowFloats * 4;
}

__device__ __forceinline__ void wait_vmcnt0() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// copy one prepared tile (NG KiB + aux) into LDS with direct global->LDS loads;
// every wave issues the same number of loads (pieces past the end re-read the
// last piece and land in the buffer's pad) so vmcnt counts are uniform
template <int NG>
__device__ __forceinline__ void load_tile(const unsigned char* __restrict__ src, unsigned char* lds_dst) {
  using G = TileGeom<NG>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int it = 0; it < G::kPerWave; ++it) {
    int k = it * 64 * kWaves + wave * 64 + lane;
    int kc = k < G::kChunks ? k : G::kChunks - 1;
    unsigned char* dst = lds_dst + (it * 64 * kWaves + wave * 64) * 16;
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + (int64_t)kc * 16),
                                     (__attribute__((address_space(3))) void*)(dst), 16, 0, 0);
  }
}

template <int DT, int NG, int NCB>
struct MmaTile {
  // acc[cb] = init + sum over the tile depth of A(tile rows) x B(query columns)
  static __device__ __forceinline__ void run(f32x16 (&acc)[NCB], const unsigned char* tile,
                                             const u32x4 (&bq)[NCB][NG], const f32x16& init, int sa,
                                             const int (&sb)[NCB]) {
    const int lane = threadIdx.x & 63;
    if constexpr (DT == DT_FP8) {
      u32x4 af[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) af[g] = *reinterpret_cast<const u32x4*>(tile + g * 1024 + lane * 16);
#pragma unroll
      for (int s = 0; s < NG / 2; ++s) {
        const u32x4& a0 = af[2 * s];
        const u32x4& a1 = af[2 * s + 1];
        i32x8 A = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const u32x4& b0 = bq[cb][2 * s];
          const u32x4& b1 = bq[cb][2 * s + 1];
          i32x8 B = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
          acc[cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, s == 0 ? init : acc[cb], 0, 0, 0, sa, 0,
                                                                     sb[cb]);
        }
      }
    } else if constexpr (DT == DT_BF16) {
      u32x4 af[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) af[g] = *reinterpret_cast<const u32x4*>(tile + g * 1024 + lane * 16);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        bf16x8 A = __builtin_bit_cast(bf16x8, af[g]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          bf16x8 B = __builtin_bit_cast(bf16x8, bq[cb][g]);
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, g == 0 ? init : acc[cb], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        u32x4 a = *reinterpret_cast<const u32x4*>(tile + g * 1024 + lane * 16);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[e]), __uint_as_float(bq[cb][g][e]),
                                                           (g == 0 && e == 0) ? init : acc[cb], 0, 0, 0);
          }
        }
      }
    }
  }
};

// merge the two lane halves' (value, row) of one query: larger value, then lower row
__device__ __forceinline__ void merge_halves(float v, int i, float& mv, int& mi) {
  float ov = __shfl_xor(v, 32);
  int oi = __shfl_xor(i, 32);
  bool take = (ov > v) || (ov == v && oi < i);
  mv = take ? ov : v;
  mi = take ? oi : i;
}

__device__ __forceinline__ void write_bin(float* __restrict__ outV, int32_t* __restrict__ outA, int64_t ldo,
                                          int64_t q, int64_t bin, float v, int idx, float sign) {
  outV[q * ldo + bin] = sign * v;
  outA[q * ldo + bin] = idx >= kSentinel ? -1 : idx;
}

template <int DT, int NG, int NCB>
__device__ __forceinline__ void run_item(const unsigned char* __restrict__ db_tiles,
                                         const unsigned char* __restrict__ q_tiles, int64_t N, int64_t L, int64_t M,
                                         int64_t q0, int64_t b0, int64_t b1, float sign, float* __restrict__ outV,
                                         int32_t* __restrict__ outA, int64_t ldo, unsigned char* lds) {
  using G = TileGeom<NG>;
  constexpr int64_t TB = (int64_t)NG * 1024 + kAuxBytes;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, ql = lane & 31;
  unsigned char* buf0 = lds;
  unsigned char* buf1 = lds + G::kLdsBytes;
  float* scratch = reinterpret_cast<float*>(lds + 2 * G::kLdsBytes) + wave * kSlowFloats;

  const int64_t r0 = bin_start(b0, N, L), r1 = bin_start(b1, N, L);
  const int64_t t_first = r0 >> 5, t_last = (r1 - 1) >> 5;
  load_tile<NG>(db_tiles + t_first * TB, buf0);

  // query fragments of this wave (tiles of 32 queries; the buffer is padded)
  const int64_t wq0 = q0 + (int64_t)wave * 32 * NCB;
  u32x4 bq[NCB][NG];
  int sb[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const unsigned char* qt = q_tiles + ((wq0 >> 5) + cb) * TB;
#pragma unroll
    for (int g = 0; g < NG; ++g) bq[cb][g] = *reinterpret_cast<const u32x4*>(qt + g * 1024 + lane * 16);
    sb[cb] = qt[NG * 1024 + 128 + ql];
  }
  const bool active = wq0 < M;

  // running bin state per column block and lane half: best value, the tile (first
  // row) it came from and the row offset inside the tile, so the per-score index
  // update only moves an inline constant
  float bv[NCB];
  int bt[NCB], bo[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    bv[cb] = -INFINITY;
    bt[cb] = kSentinel;
    bo[cb] = 0;
  }
  auto abs_index = [&](int cb) { return bt[cb] == kSentinel ? kSentinel : bt[cb] + bo[cb] + 4 * h; };
  int64_t cur_bin = b0;
  int64_t next_start = bin_start(b0 + 1, N, L);

  for (int64_t t = t_first; t <= t_last; ++t) {
    unsigned char* cur = ((t - t_first) & 1) ? buf1 : buf0;
    unsigned char* nxt = ((t - t_first) & 1) ? buf0 : buf1;
    wait_vmcnt0();
    __syncthreads();
    if (t < t_last) load_tile<NG>(db_tiles + (t + 1) * TB, nxt);
    if (!active) continue;

    const float* auxf = reinterpret_cast<const float*>(cur + NG * 1024);
    f32x16 init;
#pragma unroll
    for (int i = 0; i < 16; ++i) init[i] = auxf[h * 16 + i];
    const int sa = cur[NG * 1024 + 128 + ql];
    f32x16 acc[NCB];
    MmaTile<DT, NG, NCB>::run(acc, cur, bq, init, sa, sb);

    const int64_t t0 = t << 5;
    const int64_t lo = t0 > r0 ? t0 : r0;
    const int64_t hi = (t0 + 32) < r1 ? (t0 + 32) : r1;
    const int t0i = (int)t0;
    if (lo == t0 && hi == t0 + 32 && t0 + 32 <= next_start) {
      // the whole tile lies inside the current bin
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float before = bv[cb];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float s = acc[cb][i];
          const bool c = s > bv[cb];
          bv[cb] = c ? s : bv[cb];
          bo[cb] = c ? (8 * (i >> 2) + (i & 3)) : bo[cb];
        }
        bt[cb] = bv[cb] != before ? t0i : bt[cb];
      }
      if (t0 + 32 == next_start) {  // the bin ends with this tile
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          float mv;
          int mi;
          merge_halves(bv[cb], abs_index(cb), mv, mi);
          const int64_t q = wq0 + cb * 32 + ql;
          if (h == 0 && q < M) write_bin(outV, outA, ldo, q, cur_bin, mv, mi, sign);
          bv[cb] = -INFINITY;
          bt[cb] = kSentinel;
          bo[cb] = 0;
        }
        ++cur_bin;
        next_start = bin_start(cur_bin + 1, N, L);
      }
    } else {
      // tile crosses a bin boundary or the chunk edge: walk its rows in order
      int64_t cb2 = cur_bin, ns = next_start;
#pragma unroll
      for (int rd = 0; rd < (NCB + 1) / 2; ++rd) {
        const int cA = 2 * rd, cB = 2 * rd + 1;
        const bool hasB = cB < NCB;
        float sv = -INFINITY;
        int si = kSentinel;
        {
          float mv;
          int mi;
          merge_halves(bv[cA], abs_index(cA), mv, mi);
          if (h == 0) { sv = mv; si = mi; }
          if (hasB) {
            merge_halves(bv[cB], abs_index(cB), mv, mi);
            if (h == 1) { sv = mv; si = mi; }
          }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = 8 * (i >> 2) + 4 * h + (i & 3);
          scratch[ql * 33 + row] = acc[cA][i];
          if (hasB) scratch[32 * 33 + ql * 33 + row] = acc[cB][i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool lane_on = (h == 0) || hasB;
        const int64_t q = wq0 + (cA + h) * 32 + ql;
        cb2 = cur_bin;
        ns = next_start;
        const float* my = scratch + h * 32 * 33 + ql * 33;
        for (int jj = 0; jj < 32; ++jj) {
          const int64_t j = t0 + jj;
          if (j < lo || j >= hi) continue;
          if (j == ns) {
            if (lane_on && q < M) write_bin(outV, outA, ldo, q, cb2, sv, si, sign);
            sv = -INFINITY;
            si = kSentinel;
            ++cb2;
            ns = bin_start(cb2 + 1, N, L);
          }
          const float s = my[jj];
          if (s > sv) { sv = s; si = (int)j; }
        }
        if (hi == ns) {
          if (lane_on && q < M) write_bin(outV, outA, ldo, q, cb2, sv, si, sign);
          sv = -INFINITY;
          si = kSentinel;
          ++cb2;
          ns = cb2 < b1 ? bin_start(cb2 + 1, N, L) : r1;
        }
        // back to the per-half form: half 0 carries the open bin's state
        {
          const float vA = __shfl(sv, ql);
          const int iA = __shfl(si, ql);
          bv[cA] = h == 0 ? vA : -INFINITY;
          bt[cA] = h == 0 ? iA : kSentinel;
          bo[cA] = 0;
          if (hasB) {
            const float vB = __shfl(sv, 32 + ql);
            const int iB = __shfl(si, 32 + ql);
            bv[cB] = h == 0 ? vB : -INFINITY;
            bt[cB] = h == 0 ? iB : kSentinel;
            bo[cB] = 0;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      cur_bin = cb2;
      next_start = ns;
    }
  }
}

template <int DT, int NG, int NCB>
__global__ __launch_bounds__(256) void fused_kernel(FusedParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int64_t chunk = (int64_t)(slot / p.n_qb) * 8 + xcd;
  const int qb = slot % p.n_qb;
  if (chunk >= p.n_chunks) return;
  const int64_t b0 = chunk * p.bins_per_chunk;
  const int64_t b1 = (b0 + p.bins_per_chunk) < p.L ? (b0 + p.bins_per_chunk) : p.L;
  run_item<DT, NG, NCB>(p.db_tiles, p.q_tiles, p.N, p.L, p.M, (int64_t)qb * (kWaves * 32 * NCB), b0, b1, p.out_sign, p.binV,
                        p.binA, p.ldo, lds);
}

template <int DT, int NG, int NCB>
hipError_t launch_one(const FusedParams& p, hipStream_t s) {
  const int64_t per_xcd = ceil_div(p.n_chunks, 8);
  const int64_t grid = 8 * per_xcd * p.n_qb;
  constexpr int lb = lds_bytes<NG, NCB>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_kernel<DT, NG, NCB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lb);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  fused_kernel<DT, NG, NCB><<<dim3((unsigned)grid), dim3(64 * kWaves), lb, s>>>(p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- persistent batched form
template <int DT, int NG, int NCB>
__device__ __forceinline__ void run_group_item(const GroupDesc& gd, const WorkItem& it, unsigned char* lds) {
  run_item<DT, NG, NCB>(gd.db_tiles, gd.q_tiles, gd.N, gd.L, gd.M, (int64_t)it.qb * (kWaves * 32 * NCB), it.b0,
                        it.b1, gd.out_sign, gd.binV, gd.binA, gd.ldo, lds);
}

template <int DT>
__global__ __launch_bounds__(256) void fused_persistent_kernel(const GroupDesc* __restrict__ groups,
                                                               const WorkItem* __restrict__ items, int64_t n_items) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  for (int64_t w = blockIdx.x; w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    if (it.grp < 0) continue;  // padding slot of the per-XCD work lists
    const GroupDesc gd = groups[it.grp];
    __syncthreads();  // the previous item's LDS use is over
    switch (gd.ng * 4 + gd.ncb) {
      // BF16 depths 64, 96, 128, 256 (NG = 4, 6, 8, 16) and FP32 / FP8 equivalents
      case 4 * 4 + 1: run_group_item<DT, 4, 1>(gd, it, lds); break;
      case 4 * 4 + 2: run_group_item<DT, 4, 2>(gd, it, lds); break;
      case 6 * 4 + 1: run_group_item<DT, 6, 1>(gd, it, lds); break;
      case 6 * 4 + 2: run_group_item<DT, 6, 2>(gd, it, lds); break;
      case 8 * 4 + 1: run_group_item<DT, 8, 1>(gd, it, lds); break;
      case 8 * 4 + 2: run_group_item<DT, 8, 2>(gd, it, lds); break;
      case 16 * 4 + 1: run_group_item<DT, 16, 1>(gd, it, lds); break;
      default: break;
    }
  }
}

}  // namespace

int fused_lds_bytes(int ng, int ncb) {
  (void)ncb;
  int per_wave = (ng * 64 + kAuxBytes / 16 + 64 * kWaves - 1) / (64 * kWaves);
  return 2 * per_wave * 64 * kWaves * 16 + kWaves * kSlowFloats * 4;
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
#define X(D_, G_, C_) \
  if (dt == D_ && ng == G_ && ncb == C_) return launch_one<D_, G_, C_>(p, s);
  KNN_FUSED_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fused_persistent(int dt, const GroupDesc* d_groups, const WorkItem* d_items, int64_t n_items,
                                   int n_blocks, int max_ng, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  if (dt != DT_BF16) return hipErrorInvalidValue;  // the batched form is built for BF16 databases
  const int lb = fused_lds_bytes(max_ng, 2);
  static int attr_bytes = 0;
  if (lb > attr_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_persistent_kernel<DT_BF16>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lb);
    if (e != hipSuccess) return e;
    attr_bytes = lb;
  }
  fused_persistent_kernel<DT_BF16><<<n_blocks, 64 * kWaves, lb, s>>>(d_groups, d_items, n_items);
  return hipGetLastError();
}

}  // namespace knn
