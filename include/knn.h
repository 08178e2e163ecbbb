/*
 * knn.h -- C ABI of the MI355X (gfx950) approximate K-NN library.
 *
 * The library implements the two-kernel search of "TPU-KNN: K Nearest
 * Neighbor Search at Peak FLOP/s" (Chern et al., 2022):
 *   PartialReduce (Sec. 5, Algorithm 1): the query-database distance GEMM fused
 *     with a reduction that keeps, for each query, the best score and its row
 *     index in each of L bins, so the M x N score matrix never reaches memory;
 *   ExactRescoring (Sec. 5): the exact top-K over the M x L bin winners.
 * Scores (Sec. 2 and the appendix on Euclidean search):
 *   KNN_MIPS    <q, x>                      maximised (eq. 2)
 *   KNN_L2      |x|^2 / 2 - <q, x>          minimised (eq. l2final); returned as is,
 *                                           so |q - x|^2 = 2 * value + |q|^2
 *   KNN_COSINE  <q, x> / (|q| |x|)          maximised; cosine distance = 1 - value;
 *                                           a zero-norm row or query scores 0
 * Bins are contiguous balanced row ranges: bin b holds rows
 *   [floor(b N / L), floor((b + 1) N / L)),
 * which is Algorithm 1's ShiftRight(j, W) when N = L * 2^W.  Inside a bin the
 * lowest row index wins ties; results are ordered best first, ties by lower index.
 * Expected recall (Sec. 5.1, eq. recall) is at least ((L-1)/L)^(K-1).
 *
 * Conventions for every entry point:
 *   - Pointers named Q, X, out_*, bins_*, g, idx, dQ, dX, buf, workspace are DEVICE
 *     pointers, owned by the caller, row-major and contiguous.  FP32 data is 4-byte
 *     aligned, BF16 data 2-byte aligned, buf and workspace 16-byte aligned.
 *   - Device memory is the caller's: the library allocates none, except knn_search
 *     (the plain form, which takes raw rows and prepares them on every call).  Each call
 *     that needs memory beyond its inputs and outputs takes a `workspace` of at least the
 *     size its *_workspace_size query reports, and a prepared database lives in a buffer
 *     of knn_db_prepare_size bytes.  The handles knn_db and knn_plan are small host
 *     objects owned by the library; they point into that caller memory, which must stay
 *     valid and unchanged for their lifetime.  A workspace holds nothing between calls;
 *     calls that share one must not overlap in time (order them on one stream).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it
 *     and the call returns without synchronising, except where noted; the calls that do
 *     not synchronise may be captured into a hipGraph.
 *   - Arguments are checked before anything is enqueued.  On error the call returns
 *     a non-zero knn_status, knn_last_error() describes it (per thread), nothing is
 *     enqueued and the outputs are untouched.  No C++ exception crosses the ABI.
 *   - Sizes: 1 <= K <= L <= N <= 2^31 - 64, 1 <= D <= 256, M >= 0 (M = 0 is a no-op).
 *     Row indices are int32.
 *   - Inputs with NaN or infinity give unspecified results (they are not scanned).
 */
#ifndef KNN_MI355X_H
#define KNN_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KNN_OK = 0,
  KNN_ERR_INVALID = 1,     /* bad argument: size, pointer, enum, handle */
  KNN_ERR_UNSUPPORTED = 2, /* valid but not implemented (e.g. D > 256) */
  KNN_ERR_OOM = 3,         /* device or host allocation failed */
  KNN_ERR_HIP = 4          /* a HIP runtime call or kernel launch failed */
} knn_status;

typedef enum { KNN_MIPS = 0, KNN_L2 = 1, KNN_COSINE = 2 } knn_metric;

/* Element types.  KNN_F32 and KNN_BF16 may be input types; all three may be the
 * compute type of the distance GEMM (FP32 accumulation in every case).
 * KNN_FP8_E4M3 is the OCP E4M3 format (max 448) with one power-of-two scale per
 * row: x ~ code(x * 2^-e) * 2^e, e the smallest integer with max|x| <= 448 * 2^e. */
typedef enum { KNN_F32 = 0, KNN_BF16 = 1, KNN_FP8_E4M3 = 2 } knn_dtype;

typedef struct knn_db knn_db;     /* a prepared database (opaque) */
typedef struct knn_plan knn_plan; /* a batched search plan (opaque) */

/* ------------------------------------------------------------------ helpers (host only) */

/* Smallest L with ((L-1)/L)^(K-1) >= r (Sec. 5.1, eq. l:approx, exact inverse),
 * clamped to [K, N]; K == 1 gives 1.  Returns -1 for K < 1, N < 1 or r outside (0, 1). */
int64_t knn_bins_for_recall(int32_t K, double recall_target, int64_t N);

/* ((L-1)/L)^(K-1) (Sec. 5.1, eq. recall); NaN for K < 1 or L < 1. */
double knn_expected_recall_bound(int32_t K, int64_t L);

/* First row of bin b: floor(b N / L).  -1 for invalid arguments. */
int64_t knn_bin_start(int64_t b, int64_t N, int64_t L);

/* Static description of a status code. */
const char* knn_status_string(int32_t status);

/* Message of the last failed call on this thread ("" if none). */
const char* knn_last_error(void);

/* Number of HIP devices visible (0 without a GPU); never fails. */
int32_t knn_device_count(void);

/* ------------------------------------------------------------------ database preparation */

/* Bytes of device memory a prepared database of N rows of depth D takes (the rows
 * converted to `compute` and laid out in tiles, plus the original rows' half norms for
 * L2 or inverse norms for cosine).  0 for invalid arguments. */
size_t knn_db_prepare_size(int64_t N, int32_t D, int32_t metric, int32_t compute);

/* Prepare a database once for many searches, into the caller's buffer.  The paper
 * passes the L2 half norms precomputed (appendix on Euclidean search) and pads the depth
 * to the matrix unit's (100 -> 128 in its benchmark appendix); this call does both:
 * for cosine the rows are unit-normalised in FP32; rows are then converted to `compute`
 * (FP32 copy, BF16 round-to-nearest-even, or per-row scaled FP8 E4M3), zero-padded to
 * the MFMA depth and stored in the layout the distance kernel streams; L2 also stores
 * |x~|^2 / 2 of the converted rows.
 *   X        device, N x D, type in_dtype (KNN_F32 or KNN_BF16).  The handle keeps X's
 *            pointer for the FP32 rerank of low-precision searches: X must stay valid
 *            and unchanged for the life of the handle.
 *   buf      device, at least knn_db_prepare_size(N, D, metric, compute) bytes; holds
 *            the prepared database for the life of the handle
 *   out      receives the handle (a host object); release it with knn_db_destroy.
 * Enqueues one kernel on `stream`; no allocation of device memory, no synchronisation. */
knn_status knn_db_prepare(const void* X, int32_t in_dtype, int64_t N, int32_t D, int32_t metric, int32_t compute,
                          void* buf, size_t bytes, void* stream, knn_db** out);

/* Release the handle (not the caller's buffer). */
knn_status knn_db_destroy(knn_db* db);

/* Copy the prepared rows back to HOST buffers in plain row-major form, for tests:
 *   codes      N x D elements of the compute type (float, uint16 BF16 bits, uint8 E4M3 codes)
 *   exponents  N int32 row exponents e (FP8 only; may be NULL)
 *   half_norms N floats |x~|^2 / 2 (L2 only; may be NULL).
 * Synchronises `stream`. */
knn_status knn_db_export(const knn_db* db, void* codes, int32_t* exponents, float* half_norms,
                         void* stream);

/* ------------------------------------------------------------------ search */

/* The plain FP32 search (Sec. 2 eq. 1-2; Sec. 5: PartialReduce, Algorithm 1, then the
 * exact top-K of the bin winners): Q (M x D) against X (N x D), both FP32 device arrays.
 * L <= 0 chooses L = knn_bins_for_recall(K, 0.95, N).  Writes the best K per query,
 * best first: out_val FP32[M x K], out_idx int32[M x K].  Being the form that takes raw
 * rows, it prepares X on every call into a stream-ordered temporary from a memory pool
 * the library keeps per device (freed memory is kept for later calls until the process
 * ends); knn_db_prepare + knn_db_search is the allocation-free form. */
knn_status knn_search(const float* Q, int64_t M, const float* X, int64_t N, int32_t D, int32_t K,
                      int64_t L, int32_t metric, float* out_val, int32_t* out_idx, void* stream);

/* Search a prepared database with the options of the paper's op (App. A.1).
 *   Q          device, M x D, type q_dtype (KNN_F32 or KNN_BF16)
 *   L          bins; L <= 0 derives it from recall_target (<= 0: 0.95) by eq. l:approx
 *              (Sec. 5.1) for input_size_override rows if that is > 0, else for the
 *              database's N rows, keeping that bin density on these rows, as
 *              knn_approx_bins does: a database that is one bin-aligned shard of a
 *              longer one then gets exactly the longer one's bins (the override's use
 *              in a distributed search, App. A.1)
 *   rerank_k   0: return the top-K of the bin winners by the compute-type score;
 *              K..min(L, 1024): take the best rerank_k bin winners by the compute-type
 *              score, rescore them in FP32 from the original Q and X rows, return the
 *              best K (the precision form of the search: BF16 / FP8 GEMM + FP32 rerank)
 *   out_val/out_idx  M x K, best first (scores are FP32 rescored ones when reranking)
 *   bins_val/bins_idx optional M x L bin winners (Algorithm 1's V and A, compute-type
 *              scores in the metric's own sign); NULL to skip (the `aggregate_to_topk`
 *              option of the paper's op corresponds to out_* being used)
 *   workspace  device, >= the size knn_db_search_workspace_size reports for the same
 *              arguments (NULL allowed when that is 0)
 * No allocation, no synchronisation: may be captured into a hipGraph. */
knn_status knn_db_search(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K, int64_t L,
                         double recall_target, int64_t input_size_override, int32_t rerank_k, float* out_val,
                         int32_t* out_idx, float* bins_val, int32_t* bins_idx, void* workspace, size_t ws_bytes,
                         void* stream);

/* Workspace bytes knn_db_search needs for these arguments (with_bins: bins_val and
 * bins_idx will be given).  Host only. */
knn_status knn_db_search_workspace_size(const knn_db* db, int64_t M, int32_t K, int64_t L, double recall_target,
                                        int64_t input_size_override, int32_t rerank_k, int32_t with_bins,
                                        size_t* bytes);

/* knn_db_search for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation): the same arguments
 * without the workspace, which comes instead from a fixed device array of
 * knn_noalloc_scratch_bytes() bytes (32 MiB) that the library holds on every device it
 * runs on until the process ends.  A search whose workspace would exceed it
 * (knn_db_search_workspace_size) returns KNN_ERR_INVALID with nothing enqueued.  No
 * allocation, no synchronisation; the stream must belong to the current device.  All
 * calls on one device share that array, so calls that overlap in time on one device
 * (other streams, other threads) race: order them on one stream. */
knn_status knn_db_search_noalloc(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K, int64_t L,
                                 double recall_target, int64_t input_size_override, int32_t rerank_k,
                                 float* out_val, int32_t* out_idx, float* bins_val, int32_t* bins_idx,
                                 void* stream);
size_t knn_noalloc_scratch_bytes(void);

/* The two steps of a search exposed on their own, for callers that reuse prepared
 * queries and for timing the distance kernel alone.
 * knn_query_buffer_bytes: size of the device buffer knn_query_prepare fills for M queries.
 * knn_query_prepare: queries -> the layout the distance kernel reads (same conversion as
 *   the database: cosine normalisation, compute type, padding).  qbuf is a device buffer
 *   of at least knn_query_buffer_bytes(db, M) bytes, owned by the caller.
 * knn_partial_reduce: PartialReduce alone (Sec. 5, Algorithm 1): the M x L bin winners
 *   (bins_val FP32, bins_idx int32, device, row-major), compute-type scores in the
 *   metric's own sign; no top-K (the `aggregate_to_topk = False` form of the paper's op).
 *   bins_idx is in compact form: an entry >= 0 is the winning row; -1 means no finite
 *   score; smaller entries name a set of rows the winner is among (the kernel tracks
 *   the best of groups of its accumulators): e > -2 - 2^29: the 4 rows from
 *   s = 4 (-2 - e); -2 - 2^30 < e <= -2 - 2^29: rows s .. s+3 and s+8 .. s+11 with
 *   s = 4 (-2 - 2^29 - e); e <= -2 - 2^30: the 16 rows from s = 16 (-2 - 2^30 - e).
 * knn_resolve_rows: replaces every compact entry of idx (M x ncols, leading dimension
 *   ld, row i belonging to query i of qbuf) by the exact row: the entry's rows are
 *   rescored from the prepared rows in FP32 and the best (lowest row on ties) is kept.
 *   knn_db_search does this itself; its outputs always hold exact rows. */
size_t knn_query_buffer_bytes(const knn_db* db, int64_t M);
knn_status knn_query_prepare(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, void* qbuf,
                             size_t qbuf_bytes, void* stream);
knn_status knn_partial_reduce(const knn_db* db, const void* qbuf, int64_t M, int64_t L, float* bins_val,
                              int32_t* bins_idx, void* stream);
knn_status knn_resolve_rows(const knn_db* db, const void* qbuf, int64_t M, int64_t ncols, int32_t* idx, int64_t ld,
                            void* stream);

/* ------------------------------------------------------------------ batched search */

/* One query batch of a batched plan: M_b queries (device, M_b x D_db, FP32 or BF16
 * as q_dtype) against database `db` (an index into the plan's database list),
 * K_b results written to out_val/out_idx (device, M_b x K_b). */
typedef struct {
  const void* Q;
  int64_t M;
  int32_t db;
  int32_t K;
  float* out_val;
  int32_t* out_idx;
} knn_batch;

/* Batched search (not in the paper: many uneven query batches against several
 * databases in one persistent launch).  Three steps:
 * knn_plan_create: host only.  Plans `nb` uneven query batches against `ndb` prepared
 *   databases (BF16).  The batch pointers are bound now: every run reads the queries
 *   from, and writes the results to, the same buffers.  For each database the plan picks
 *   L >= knn_bins_for_recall(max K, recall_target, N) (more bins than that when one
 *   bin's rows would not fit the 2 MiB that a group of workgroups streams through an
 *   XCD's L2; more bins never lower the expected recall) and the kernel tiling by a fixed
 *   heuristic, or with tune != 0 by timing candidates in knn_plan_setup (the autotuner),
 *   taking earlier choices from the JSON cache file `cache_path` (NULL: no cache) when
 *   they were made for the same device, database shape, batch sizes, K and recall bound
 *   and are valid for this plan.
 * knn_plan_workspace_size: host only; the device bytes knn_plan_setup needs (covering
 *   every choice the autotuner may try).
 * knn_plan_setup: lays the plan out in the caller's workspace (prepared queries, bins,
 *   the device work list), runs the autotuner if requested (it times candidates on
 *   `stream` with hipEvents and writes the cache) and uploads the work list.
 *   Synchronises `stream`.  The workspace must stay valid for the life of the plan. */
knn_status knn_plan_create(knn_db* const* dbs, int32_t ndb, const knn_batch* batches, int32_t nb,
                           int32_t q_dtype, double recall_target, int32_t tune, const char* cache_path,
                           knn_plan** out);
knn_status knn_plan_workspace_size(const knn_plan* plan, size_t* bytes);
knn_status knn_plan_setup(knn_plan* plan, void* workspace, size_t ws_bytes, void* stream);

/* Run every batch of the plan: one query-preparation launch, a one-workgroup launch
 * that zeroes the persistent kernel's 8 item counters (held in the workspace), one
 * persistent distance + bin-reduce launch over a device work list that covers all
 * batches and databases, one top-K launch and one launch that resolves the winners'
 * rows.  No allocation, no memset, no host synchronisation: may be captured into a
 * hipGraph.  Runs on one stream at a time (the counters and bins are the plan's).
 * KNN_ERR_INVALID before knn_plan_setup. */
knn_status knn_search_batched(knn_plan* plan, void* stream);

/* Scheduling option (not in the paper): database groups with at least `min_items`
 * (query block, chunk) work items run as distance launches of their own, with the
 * kernel specialised for their depth, before the persistent launch that the smaller
 * groups share (all of it still one capturable sequence on one stream).  0, the
 * default, keeps every group in the one persistent launch.  Host only; takes effect at
 * the next knn_plan_setup (the plan must be set up again).  KNN_ERR_INVALID for a NULL
 * plan or min_items < 0. */
knn_status knn_plan_set_own_launches(knn_plan* plan, int64_t min_items);

/* The plan's per-database choices: L, query-block width and rows per work item
 * (host arrays of length ndb; any may be NULL). */
knn_status knn_plan_info(const knn_plan* plan, int64_t* L, int32_t* qblock, int64_t* chunk_rows);

/* Release the plan (not the caller's workspace). */
knn_status knn_plan_destroy(knn_plan* plan);

/* ------------------------------------------------------------------ approx_max_k on scores */

/* The number of bins the op below uses for a slice of n scores when L is not given
 * (App. A.1, the op's options): L_eval = knn_bins_for_recall(K, recall_target, n_eval)
 * with n_eval = input_size_override if > 0, else n.  With an override the slice is
 * read as a part of a longer one (a shard of a sharded reduction) and gets the same
 * bin density: L = ceil(L_eval * n / n_eval).  The result is clamped to [K, n].
 * Returns -1 for n < 1, K < 1, K > n or recall_target outside (0, 1). */
int64_t knn_approx_bins(int64_t n, int32_t K, double recall_target, int64_t input_size_override);

/* PartialReduce (Sec. 5, Algorithm 1) over a score matrix the caller already has,
 * without the distance GEMM, optionally followed by the exact top-K (ExactRescoring):
 * the approx_max_k / approx_min_k op with the options of App. A.1.
 *   scores         device, rows x cols, row-major with leading dimension ld >= cols
 *                  (element (i, j) at scores[i * ld + j]), type dtype (KNN_F32 or
 *                  KNN_BF16), aligned to its element size
 *   reduction_dim  1 (or -1, the last dimension): each row is a slice of n = cols
 *                  scores, B = rows slices; 0: each column is a slice of n = rows
 *                  scores, B = cols slices
 *   K              results per slice, 1 <= K <= n (K <= 1024 when aggregating)
 *   L              bins per slice, K <= L <= n; L <= 0 derives it from recall_target
 *                  and input_size_override (knn_approx_bins)
 *   minimize       0: larger is better (approx_max_k); 1: smaller (approx_min_k)
 *   aggregate_to_topk
 *                  1: out_val/out_idx receive the best K bin winners of each slice,
 *                     best first, ties by lower index;
 *                  0: they receive all L bin winners of each slice (bin b holds slice
 *                     positions [floor(b n / L), floor((b + 1) n / L)); the lowest
 *                     position wins ties)
 *   out_val, out_idx  device FP32 and int32, laid out like the input with the reduced
 *                  dimension replaced by the result count R (K or L): B x R row-major
 *                  for reduction_dim 1, R x B row-major for reduction_dim 0.  Indices
 *                  are positions along the reduced dimension; values are the scores
 *                  widened to FP32 (a -0 score may come back as +0).
 *   workspace      device, >= the size knn_approx_workspace_size reports (the bins of
 *                  every slice when aggregating, else 0 and NULL allowed)
 * Bit-exact: no arithmetic is done on the scores.  B = 0 is a no-op.  No allocation, no
 * synchronisation. */
knn_status knn_approx_top_k(const void* scores, int32_t dtype, int64_t rows, int64_t cols, int64_t ld,
                            int32_t reduction_dim, int32_t K, double recall_target, int64_t input_size_override,
                            int64_t L, int32_t minimize, int32_t aggregate_to_topk, float* out_val,
                            int32_t* out_idx, void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes of knn_approx_top_k for the same arguments (host only). */
knn_status knn_approx_workspace_size(int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int32_t reduction_dim,
                                     int32_t K, double recall_target, int64_t input_size_override, int64_t L,
                                     int32_t minimize, int32_t aggregate_to_topk, size_t* bytes);

/* ------------------------------------------------------------------ backward */

/* Gradient of sum_{i,k} g[i,k] * score(q_i, x_{idx[i,k]}) with the selection held
 * fixed (the retrieved indices are constants):
 *   MIPS:    dQ_i = sum_k g_ik x_j           dX_j += sum g_ik q_i
 *   L2:      dQ_i = -sum_k g_ik x_j          dX_j += sum g_ik (x_j - q_i)
 *   COSINE:  dQ_i = sum_k g_ik (x_j/(|q||x|) - c q_i/|q|^2)
 *            dX_j += sum g_ik (q_i/(|q||x|) - c x_j/|x|^2),   c the cosine score.
 *   g    device FP32 M x K;  idx device int32 M x K (entries outside [0, N) are skipped)
 *   Q, X device, in_dtype (KNN_F32 or KNN_BF16), M x D and N x D
 *   dQ   device FP32 M x D, overwritten
 *   dX   device FP32 N x D, ACCUMULATED with FP32 atomics (zero it first); NULL to skip. */
knn_status knn_backward(const float* g, const int32_t* idx, const void* Q, const void* X, int32_t in_dtype,
                        int64_t M, int64_t N, int32_t D, int32_t K, int32_t metric, float* dQ, float* dX,
                        void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KNN_MI355X_H */
