// knn_internal.h -- declarations shared by the host API and the HIP kernels.
//
// Prepared-row layout (databases and queries alike).  Rows are grouped in tiles
// of 32.  A tile holds NG*1 KiB of row data followed by a 256-byte aux block.
// The row data is cut into 16-byte pieces: piece (r, g, hf) holds dimensions
//   g*2E + hf*E + [0, E) of tile row r, E = 16 bytes / element size
//   (FP32: 4, BF16: 8, FP8: 16 elements), g < NG, hf < 2,
// and is stored at byte piece_offset(r, g, hf) = (r/4)*NG*128 + g*128 + hf*64 + (r%4)*16:
// each group of 4 consecutive rows is one contiguous block of NG*128 bytes (what
// the resolve step reads for a 4-row winner).  The distance kernel copies a tile to
// LDS so that LDS piece [g][l] (l = 0..63) is piece (l % 32, g, l / 32): one 64-lane
// 16-byte LDS load of group g is then exactly one MFMA A (or B) operand fragment of
// the 32x32 matrix instructions (two consecutive groups for the FP8 32x32x64 step).
//   aux bytes [0,128):   float init[2][16]; init[h][i] = -|x~_r|^2/2 (L2, else 0) for
//                        row r = 8*(i/4) + 4*h + i%4, the row that accumulator i of a
//                        lane in half h holds in the 32x32 MFMA output layout;
//   aux bytes [128,160): E8M0 scale byte (e + 127) of each row (FP8), 127 otherwise.
// Padding rows (beyond N or M) are zero with init 0 and scale byte 127.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>
#include <stdint.h>

namespace knn {

enum { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };
enum { MET_MIPS = 0, MET_L2 = 1, MET_COSINE = 2 };

constexpr int kTileRows = 32;
constexpr int kAuxBytes = 256;
constexpr int kWaves = 4;             // waves per workgroup of the distance kernel
constexpr int kMaxDpad = 256;
// most rows of a database (or scores along a reduced dimension): the kernels do row
// arithmetic in 32 bits and look up to a 32-row tile (or a 32-score lane chunk) ahead
constexpr int64_t kMaxRows = (int64_t(1) << 31) - 64;

__host__ __device__ inline int elem_bytes(int dt) { return dt == DT_F32 ? 4 : (dt == DT_BF16 ? 2 : 1); }
// padded depth: a multiple of one fragment group pair (32 bytes per row) and of the MFMA K step
__host__ __device__ inline int dpad_for(int D, int dt) {
  int step = dt == DT_FP8 ? 64 : 32;
  return ((D + step - 1) / step) * step;
}
__host__ __device__ inline int groups_for(int dpad, int dt) { return dpad * elem_bytes(dt) / 32; }
__host__ __device__ inline int64_t tile_bytes(int ng) { return (int64_t)ng * 1024 + kAuxBytes; }
// byte offset of piece (row r of the tile, group g, half hf) inside a tile
__host__ __device__ inline int piece_offset(int r, int g, int hf, int ng) {
  return (r >> 2) * ng * 128 + g * 128 + hf * 64 + (r & 3) * 16;
}
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// first row of bin b (contiguous balanced bins)
inline int64_t bin_start_host(int64_t b, int64_t N, int64_t L) {
  return (int64_t)(((__int128)b * N) / L);
}

// ---- preparation: rows (FP32 or BF16, row-major) -> prepared tiles
// orig_half_norm: optional |x|^2/2 of the ORIGINAL rows in FP32 (rerank of L2)
// orig_rnorm:     optional 1/|x| of the ORIGINAL rows in FP32 (rerank of cosine)
hipError_t launch_prepare(const void* src, int in_dt, int64_t rows, int D, int metric, int compute,
                          bool database, unsigned char* tiles, int64_t n_tiles, float* orig_half_norm,
                          float* orig_rnorm, hipStream_t s);

// batched query preparation: row r of the concatenated query list comes from
// src_ptrs[seg][r - seg_row0[seg]]; segments sorted by seg_row0.
struct QSeg {
  const void* src;       // rows of this segment (NULL for a padding segment)
  int64_t first;         // index of the segment's first row in the global launch range
  int64_t rows;          // valid source rows (rows past it up to the next segment are padding)
  int64_t dst_row0;      // destination row of the segment's first row in `tiles`
  int32_t D, ng, metric, pad_;
  unsigned char* tiles;  // destination tile array (the group's query tiles)
};
hipError_t launch_prepare_segments(const QSeg* d_segs, int nseg, int64_t total_rows, int in_dt, int compute,
                                   hipStream_t s);

// ---- distance GEMM + bin reduce (Algorithm 1), one launch over (query block, bin chunk)
struct FusedParams {
  const unsigned char* db_tiles;
  const unsigned char* q_tiles;
  int64_t N, L, M;
  int64_t bins_per_chunk, n_chunks;
  int32_t n_qb;       // query blocks of kWaves*32*ncb queries
  float out_sign;     // +1, or -1 for L2 (the kernel maximises <q,x> - |x|^2/2)
  float* binV;        // [M x ldo] bin winners in the metric's own sign
  int32_t* binA;
  int64_t ldo;
  int32_t zero_init;  // the accumulators start from 0 (MIPS, cosine: no half norms)
};
// ncb: 32-query column blocks per wave (1 or 2)
hipError_t launch_fused(int dt, int ng, int ncb, const FusedParams& p, hipStream_t s);
bool fused_supported(int dt, int ng, int ncb);
int fused_lds_bytes(int dt, int ng, int ncb);

// ---- persistent batched distance kernel
struct WorkItem {      // one (database group, query block, bin chunk) unit
  int32_t grp;         // database group index
  int32_t qb;          // query block within the group
  int64_t b0, b1;      // bin range
};
struct GroupDesc {     // all queries against one database, concatenated
  const unsigned char* db_tiles;
  const unsigned char* q_tiles;
  int64_t N, L, M;     // M = total queries of the group
  float out_sign;
  float* binV;
  int32_t* binA;
  int64_t ldo;
  int32_t ng, ncb;
  int32_t zero_init, pad_;  // as FusedParams::zero_init
};
// The items are 8 lists of n_items / 8, one per XCD (workgroup b runs on XCD b % 8);
// the workgroups of an XCD take its items in list order through the counter
// claim[xcd], which the launch resets first (a kernel, not a memset: graph-safe).
// lds_bytes_needed: the largest fused_lds_bytes() over the groups the items touch.
hipError_t launch_fused_persistent(int dt, const GroupDesc* d_groups, const WorkItem* d_items, int64_t n_items,
                                   unsigned* d_claim, int n_blocks, int lds_bytes_needed, hipStream_t s);

// Raise a kernel's dynamic LDS limit to at least `bytes` on the current device (once
// per kernel, device and size; function attributes are per device).
inline hipError_t ensure_dynamic_lds(const void* fn, int bytes) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> granted;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  int& cur = granted[{fn, dev}];
  if (cur >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) cur = bytes;
  return e;
}

// ---- exact top-K over candidate lists (ExactRescoring)
// row r: candidates V[r*ldv + c], A[r*ldv + c] for c < n, in the metric's own sign.
// out: K per row, best first (smallest first when `minimize`), ties by lower index.
// es / eo: element strides of the candidates and of the outputs within a row
// (1 for row-major lists; the column count for lists laid out down the columns).
hipError_t launch_select(const float* V, const int32_t* A, int64_t rows, int64_t n, int64_t ldv, int K,
                         bool minimize, float* out_val, int32_t* out_idx, int64_t ldout, hipStream_t s,
                         int64_t es = 1, int64_t eo = 1);

// per-row descriptors (batched select)
struct SelRow {
  const float* V;
  const int32_t* A;
  int64_t n;
  int32_t K;
  int32_t minimize;
  float* out_val;
  int32_t* out_idx;
  // for resolving 4-row group winners of this row's output
  const unsigned char* q_tiles;
  const unsigned char* db_tiles;
  int64_t q_row;
  int32_t ng, pad_;
};
hipError_t launch_select_rows(const SelRow* d_rows, int64_t rows, int max_K, hipStream_t s);

// ---- exact rows for bin winners recorded as 4-row groups (codes <= -2, see
// knn_fused.hip): codes[i*ld + c] for i < rows, c < cols, query i of q_tiles
hipError_t launch_resolve(int dt, int32_t* codes, int64_t rows, int64_t cols, int64_t ld,
                          const unsigned char* q_tiles, const unsigned char* db_tiles, int ng, hipStream_t s);
hipError_t launch_resolve_rows(int dt, const SelRow* d_rows, int64_t rows, hipStream_t s);

// ---- PartialReduce over a caller's score matrix (rows x cols, leading dimension ld,
// FP32 or BF16).  dim 1: each row is a slice, bins out B x L (B = rows, n = cols);
// dim 0: each column is a slice, bins out L x B (B = cols, n = rows).  1 <= L <= n.
hipError_t launch_approx_bins(const void* S, int dt, int64_t rows, int64_t cols, int64_t ld, int dim, int64_t L,
                              bool minimize, float* outV, int32_t* outA, hipStream_t s);

// ---- FP32 rerank of Kr candidates per query from the original rows
hipError_t launch_rerank(const int32_t* cand, int64_t M, int Kr, const void* Q, int q_dt, const void* X,
                         int x_dt, int D, int metric, const float* x_half_norm, const float* x_rnorm, int K,
                         float* out_val, int32_t* out_idx, hipStream_t s);

// ---- backward
hipError_t launch_backward(const float* g, const int32_t* idx, const void* Q, const void* X, int dt, int64_t M,
                           int64_t N, int D, int K, int metric, float* dQ, float* dX, hipStream_t s);

}  // namespace knn
