// knn_api.cpp -- the C ABI (include/knn.h): argument checks, buffer management,
// launch sequencing, the batched plan and its autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/knn.h"
#include "knn_internal.h"

using namespace knn;

namespace {

thread_local std::string g_last_error;

knn_status fail(knn_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
knn_status fail(knn_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

knn_status hip_fail(hipError_t e, const char* what) {
  return fail(KNN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool valid_metric(int32_t m) { return m == KNN_MIPS || m == KNN_L2 || m == KNN_COSINE; }
bool valid_in(int32_t t) { return t == KNN_F32 || t == KNN_BF16; }
bool valid_compute(int32_t t) { return t == KNN_F32 || t == KNN_BF16 || t == KNN_FP8_E4M3; }

knn_status check_sizes(int64_t M, int64_t N, int32_t D, int32_t K, int64_t L) {
  if (M < 0) return fail(KNN_ERR_INVALID, "M must be >= 0 (got %lld)", (long long)M);
  // rows of a 32-row tile plus 32 stay below 2^31 in the distance kernel's 32-bit row arithmetic
  if (N < 1 || N > kMaxRows)
    return fail(KNN_ERR_INVALID, "N must be in [1, 2^31 - 64] (got %lld)", (long long)N);
  if (D < 1) return fail(KNN_ERR_INVALID, "D must be >= 1 (got %d)", D);
  if (D > kMaxDpad) return fail(KNN_ERR_UNSUPPORTED, "D must be <= %d (got %d)", kMaxDpad, D);
  if (K < 1 || K > 1024) return fail(KNN_ERR_INVALID, "K must be in [1, 1024] (got %d)", K);
  if (L < K || L > N)
    return fail(KNN_ERR_INVALID, "need K <= L <= N (K=%d, L=%lld, N=%lld)", K, (long long)L, (long long)N);
  return KNN_OK;
}

int pick_ncb(int dt, int ng, int64_t M) {
  // two 32-query column blocks per wave when there are enough queries and the
  // query fragments fit next to the accumulators
  int ncb = (M > 128) ? 2 : 1;
  if (!fused_supported(dt, ng, ncb)) ncb = 1;
  return ncb;
}

// bins per work item: enough items to fill the chip, at least ~256 rows per item
// The workgroups that share a bin chunk run together on one XCD and stream its
// tiles through that XCD's 4 MB L2; a chunk of at most this many prepared bytes
// stays resident while they do (larger chunks let them drift apart and re-read).
constexpr double kChunkBytes = 2.0 * 1024 * 1024;

double row_bytes(int ng) { return double(tile_bytes(ng)) / kTileRows; }

// bins per work item: about target_items items in all, at least 256 rows, and at
// most kChunkBytes of prepared rows (unless one bin is larger)
int64_t pick_bins_per_chunk(int64_t N, int64_t L, int64_t n_qb, int ng, int64_t target_items = 8192) {
  const double bin_rows = double(N) / double(L);
  int64_t want_chunks = std::max<int64_t>(1, ceil_div(target_items, std::max<int64_t>(1, n_qb)));
  int64_t bpc = std::max<int64_t>(1, L / want_chunks);
  int64_t min_bpc = std::max<int64_t>(1, (int64_t)std::ceil(256.0 / bin_rows));
  int64_t max_bpc = std::max<int64_t>(1, (int64_t)(kChunkBytes / (bin_rows * row_bytes(ng))));
  bpc = std::max(bpc, min_bpc);
  bpc = std::min(bpc, std::max(max_bpc, min_bpc));
  // whole 16-bin output windows of the distance kernel: item edges on window edges
  // (or at least on 4-bin boundaries, which its 16-byte stores still cover)
  if (bpc >= 16)
    bpc = bpc / 16 * 16;
  else if (bpc >= 4)
    bpc = bpc / 4 * 4;
  return std::min<int64_t>(L, bpc);
}

// Smallest L whose bins each fit in one L2-resident chunk (never above N/32: bins
// keep at least one tile of rows).  Used by batched plans, which may choose more
// bins than the recall target needs: more bins never lower the expected recall.
int64_t bins_for_l2(int64_t N, int ng) {
  const int64_t l = (int64_t)std::ceil(double(N) * row_bytes(ng) / kChunkBytes);
  return std::max<int64_t>(1, std::min<int64_t>(l, N / kTileRows));
}

// Stream-ordered temporaries come from a library-owned memory pool per device that
// keeps freed blocks for reuse (release threshold: unlimited), so repeated searches do
// not hand large temporaries back to the driver at every synchronisation and fetch
// them again on the next call.
hipError_t library_pool(hipMemPool_t* out) {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipMemPoolProps props = {};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  e = hipMemPoolCreate(&pool, &props);
  if (e != hipSuccess) return e;
  uint64_t keep = UINT64_MAX;
  e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) return e;
  pools[dev] = pool;
  *out = pool;
  return hipSuccess;
}

struct DevBuf {  // stream-ordered temporary from the library pool
  void* p = nullptr;
  hipStream_t s = nullptr;
  hipError_t alloc(size_t bytes, hipStream_t st) {
    s = st;
    hipMemPool_t pool;
    if (library_pool(&pool) != hipSuccess) {  // no pool support: the device's default pool
      (void)hipGetLastError();
      return hipMallocAsync(&p, std::max<size_t>(bytes, 256), st);
    }
    return hipMallocFromPoolAsync(&p, std::max<size_t>(bytes, 256), pool, st);
  }
  ~DevBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

}  // namespace

// --------------------------------------------------------------------------- handles
// A prepared database lives in caller memory (knn_db_prepare); the handle is a host
// object that only points into it.
struct knn_db {
  int32_t in_dt, compute, metric, D, dpad, ng;
  int64_t N, n_tiles;
  unsigned char* tiles = nullptr;
  float* orig_half_norm = nullptr;  // L2: |x|^2/2 of the original rows (rerank)
  float* orig_rnorm = nullptr;      // cosine: 1/|x| of the original rows (rerank)
  const void* X = nullptr;          // caller's rows (not owned)
};

struct GroupPlan {  // all batches against one database
  int32_t db;
  int64_t M = 0, L = 0, L_min = 0, bins_per_chunk = 0, n_qb = 0, n_chunks = 0, q_tiles_n = 0;
  int32_t ncb = 1, K_max = 1;
  bool tune = false;  // still to be tuned in knn_plan_setup
  bool own = false;   // runs as a launch of its own (bind_plan; knn_plan_set_own_launches)
  unsigned char* q_tiles = nullptr;  // inside the bound workspace
  float* binV = nullptr;
  int32_t* binA = nullptr;
};

struct knn_plan {
  std::vector<knn_db*> dbs;
  std::vector<knn_batch> batches;
  std::vector<GroupPlan> groups;
  int32_t q_dtype = KNN_F32, compute = KNN_BF16;
  std::string cache_path;
  int64_t total_q_rows = 0, n_items = 0, n_sel_rows = 0;
  int n_blocks = 0, max_ng = 0, n_segs = 0, max_K = 1, lds_bytes = 0;
  int64_t own_launch_items = 0;  // groups with this many work items launch alone (0: never)
  bool bound = false;  // knn_plan_setup succeeded
  // descriptors: built on the host, uploaded into the workspace
  std::vector<QSeg> segs;
  std::vector<GroupDesc> gds;
  std::vector<WorkItem> items;
  std::vector<SelRow> sel;
  QSeg* d_segs = nullptr;
  GroupDesc* d_groups = nullptr;
  WorkItem* d_items = nullptr;
  unsigned* d_claim = nullptr;  // the persistent kernel's 8 per-XCD item counters
  SelRow* d_sel = nullptr;
  float* tune_val = nullptr;  // autotuner's top-K output
  int32_t* tune_idx = nullptr;
};

// --------------------------------------------------------------------------- helpers
extern "C" int64_t knn_bins_for_recall(int32_t K, double r, int64_t N) {
  if (K < 1 || N < 1 || !(r > 0.0 && r < 1.0)) return -1;
  int64_t L;
  if (K == 1) {
    L = 1;
  } else {
    double x = 1.0 / (1.0 - std::pow(r, 1.0 / (K - 1)));
    L = (int64_t)std::ceil(x);
    while (L > 1 && std::pow((double)(L - 2) / (double)(L - 1), K - 1) >= r) --L;
    while (std::pow((double)(L - 1) / (double)L, K - 1) < r) ++L;
  }
  L = std::max<int64_t>(L, K);
  return std::min<int64_t>(L, N);
}

extern "C" double knn_expected_recall_bound(int32_t K, int64_t L) {
  if (K < 1 || L < 1) return NAN;
  return std::pow((double)(L - 1) / (double)L, K - 1);
}

extern "C" int64_t knn_bin_start(int64_t b, int64_t N, int64_t L) {
  if (N < 1 || L < 1 || b < 0 || b > L) return -1;
  return bin_start_host(b, N, L);
}

extern "C" const char* knn_status_string(int32_t s) {
  switch (s) {
    case KNN_OK: return "ok";
    case KNN_ERR_INVALID: return "invalid argument";
    case KNN_ERR_UNSUPPORTED: return "unsupported";
    case KNN_ERR_OOM: return "out of memory";
    case KNN_ERR_HIP: return "HIP error";
    default: return "unknown status";
  }
}

extern "C" const char* knn_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t knn_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

// --------------------------------------------------------------------------- database
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Caller memory of a prepared database: the tiles, then (L2 / cosine) one float per
// row of the original rows' half norms / inverse norms.
struct DbLayout {
  size_t tiles = 0, aux = 0, total = 0;
};

DbLayout db_layout(int64_t N, int32_t D, int32_t metric, int32_t compute) {
  DbLayout l;
  const int ng = groups_for(dpad_for(D, compute), compute);
  l.tiles = 0;
  l.aux = align_up((size_t)(ceil_div(N, kTileRows) * tile_bytes(ng)));
  l.total = l.aux + (metric == KNN_MIPS ? 0 : align_up(sizeof(float) * (size_t)N));
  return l;
}

knn_status check_db_args(int32_t in_dtype, int64_t N, int32_t D, int32_t metric, int32_t compute) {
  if (!valid_in(in_dtype)) return fail(KNN_ERR_INVALID, "in_dtype must be KNN_F32 or KNN_BF16");
  if (!valid_compute(compute)) return fail(KNN_ERR_INVALID, "bad compute dtype %d", compute);
  if (!valid_metric(metric)) return fail(KNN_ERR_INVALID, "bad metric %d", metric);
  if (N < 1 || N > kMaxRows) return fail(KNN_ERR_INVALID, "N must be in [1, 2^31 - 64]");
  if (D < 1) return fail(KNN_ERR_INVALID, "D must be >= 1");
  if (D > kMaxDpad) return fail(KNN_ERR_UNSUPPORTED, "D must be <= %d", kMaxDpad);
  return KNN_OK;
}

}  // namespace

extern "C" size_t knn_db_prepare_size(int64_t N, int32_t D, int32_t metric, int32_t compute) {
  if (check_db_args(KNN_F32, N, D, metric, compute) != KNN_OK) return 0;
  return db_layout(N, D, metric, compute).total;
}

extern "C" knn_status knn_db_prepare(const void* X, int32_t in_dtype, int64_t N, int32_t D, int32_t metric,
                                     int32_t compute, void* buf, size_t bytes, void* stream, knn_db** out) {
  g_last_error.clear();
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  knn_status st = check_db_args(in_dtype, N, D, metric, compute);
  if (st != KNN_OK) return st;
  if (!X) return fail(KNN_ERR_INVALID, "X is NULL");
  if (!buf) return fail(KNN_ERR_INVALID, "buf is NULL");
  if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return fail(KNN_ERR_INVALID, "buf must be 16-byte aligned");
  const DbLayout lay = db_layout(N, D, metric, compute);
  if (bytes < lay.total)
    return fail(KNN_ERR_INVALID, "buf too small (%zu < %zu bytes, see knn_db_prepare_size)", bytes, lay.total);
  auto* db = new (std::nothrow) knn_db();
  if (!db) return fail(KNN_ERR_OOM, "host allocation");
  db->in_dt = in_dtype;
  db->compute = compute;
  db->metric = metric;
  db->D = D;
  db->dpad = dpad_for(D, compute);
  db->ng = groups_for(db->dpad, compute);
  db->N = N;
  db->n_tiles = ceil_div(N, kTileRows);
  db->X = X;
  unsigned char* base = static_cast<unsigned char*>(buf);
  db->tiles = base + lay.tiles;
  if (metric == KNN_L2) db->orig_half_norm = reinterpret_cast<float*>(base + lay.aux);
  if (metric == KNN_COSINE) db->orig_rnorm = reinterpret_cast<float*>(base + lay.aux);
  const hipError_t e = launch_prepare(X, in_dtype, N, D, metric, compute, true, db->tiles, db->n_tiles,
                                      db->orig_half_norm, db->orig_rnorm, (hipStream_t)stream);
  if (e != hipSuccess) {
    delete db;
    return hip_fail(e, "database preparation");
  }
  *out = db;
  return KNN_OK;
}

extern "C" knn_status knn_db_destroy(knn_db* db) {
  delete db;  // the prepared rows are the caller's memory
  return KNN_OK;
}

extern "C" knn_status knn_db_export(const knn_db* db, void* codes, int32_t* exponents, float* half_norms,
                                    void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  if (!codes) return fail(KNN_ERR_INVALID, "codes is NULL");
  const int64_t TB = tile_bytes(db->ng);
  std::vector<unsigned char> host((size_t)(db->n_tiles * TB));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "sync");
  HIP_TRY(hipMemcpy(host.data(), db->tiles, host.size(), hipMemcpyDeviceToHost), "copy prepared rows");
  const int es = elem_bytes(db->compute), E = 16 / es;
  unsigned char* out = (unsigned char*)codes;
  for (int64_t r = 0; r < db->N; ++r) {
    const unsigned char* tb = host.data() + (r >> 5) * TB;
    const int rr = (int)(r & 31);
    for (int d = 0; d < db->D; ++d) {
      const int g = d / (2 * E), hf = (d % (2 * E)) / E, k = d % E;
      memcpy(out + ((size_t)r * db->D + d) * es, tb + piece_offset(rr, g, hf, db->ng) + k * es, es);
    }
    const unsigned char* aux = tb + db->ng * 1024;
    if (exponents) exponents[r] = (int32_t)aux[128 + rr] - 127;
    if (half_norms) {
      const int half = (rr >> 2) & 1, idx = 4 * (rr >> 3) + (rr & 3);
      float v;
      memcpy(&v, aux + (half * 16 + idx) * 4, 4);
      half_norms[r] = -v;
    }
  }
  return KNN_OK;
}

// --------------------------------------------------------------------------- search core
namespace {

// Workspace of one search: the prepared queries, the M x L bin winners (unless the
// caller takes them), the rerank candidates.  Offsets are 256-byte aligned.
struct SearchLayout {
  int ncb = 1;
  int64_t n_qb = 0, q_tiles_n = 0, bpc = 0, n_chunks = 0;
  size_t q = 0, bv = 0, ba = 0, cv = 0, ci = 0, total = 0;
};

SearchLayout search_layout(const knn_db* db, int64_t M, int64_t L, int32_t rerank_k, bool bins_given) {
  SearchLayout l;
  if (M == 0) return l;
  l.ncb = pick_ncb(db->compute, db->ng, M);
  const int64_t QB = (int64_t)kWaves * 32 * l.ncb;
  l.n_qb = ceil_div(M, QB);
  l.q_tiles_n = l.n_qb * QB / kTileRows;
  l.bpc = pick_bins_per_chunk(db->N, L, l.n_qb, db->ng);
  l.n_chunks = ceil_div(L, l.bpc);
  size_t off = 0;
  l.q = off;
  off += align_up((size_t)(l.q_tiles_n * tile_bytes(db->ng)));
  if (!bins_given) {
    l.bv = off;
    off += align_up(sizeof(float) * (size_t)(M * L));
    l.ba = off;
    off += align_up(sizeof(int32_t) * (size_t)(M * L));
  }
  if (rerank_k > 0) {
    l.cv = off;
    off += align_up(sizeof(float) * (size_t)(M * rerank_k));
    l.ci = off;
    off += align_up(sizeof(int32_t) * (size_t)(M * rerank_k));
  }
  l.total = off;
  return l;
}

// L of a search: given, or the smallest meeting the recall target (eq. l:approx) for the
// database's rows or, with an input-size override, for that many rows at the same bin
// density (the database is then one shard of a longer one).  -1 if invalid.
int64_t resolve_bins(int64_t N, int32_t K, int64_t L, double recall_target, int64_t input_size_override) {
  if (L > 0) return L;
  const double r = recall_target > 0.0 ? recall_target : 0.95;
  return knn_approx_bins(N, K, r, input_size_override);
}

knn_status check_search(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K, int64_t L,
                        int32_t rerank_k, const float* out_val, const int32_t* out_idx, const float* bins_val,
                        const int32_t* bins_idx) {
  knn_status st = check_sizes(M, db->N, db->D, K, L);
  if (st != KNN_OK) return st;
  if (!valid_in(q_dtype)) return fail(KNN_ERR_INVALID, "q_dtype must be KNN_F32 or KNN_BF16");
  if (M > 0 && (!Q || !out_val || !out_idx)) return fail(KNN_ERR_INVALID, "Q, out_val and out_idx must be non-NULL");
  if ((bins_val == nullptr) != (bins_idx == nullptr))
    return fail(KNN_ERR_INVALID, "bins_val and bins_idx must both be given or both be NULL");
  if (rerank_k != 0 && (rerank_k < K || rerank_k > L || rerank_k > 1024))
    return fail(KNN_ERR_INVALID, "rerank_k must be 0 or in [K, min(L, 1024)] (got %d)", rerank_k);
  if ((int64_t)M * L >= (int64_t(1) << 40)) return fail(KNN_ERR_UNSUPPORTED, "M * L too large");
  return KNN_OK;
}

}  // namespace

// every buffer comes from `ws` (search_layout's size, checked by the caller)
static knn_status search_core(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K, int64_t L,
                              int32_t rerank_k, float* out_val, int32_t* out_idx, float* bins_val,
                              int32_t* bins_idx, unsigned char* ws, hipStream_t s) {
  if (M == 0) return KNN_OK;
  const int dt = db->compute, ng = db->ng;
  const SearchLayout lay = search_layout(db, M, L, rerank_k, bins_val != nullptr);
  unsigned char* qbuf = ws + lay.q;
  float* binV = bins_val ? bins_val : reinterpret_cast<float*>(ws + lay.bv);
  int32_t* binA = bins_idx ? bins_idx : reinterpret_cast<int32_t*>(ws + lay.ba);
  HIP_TRY(launch_prepare(Q, q_dtype, M, db->D, db->metric, dt, false, qbuf, lay.q_tiles_n, nullptr, nullptr, s),
          "query preparation");
  FusedParams p{};
  p.db_tiles = db->tiles;
  p.q_tiles = qbuf;
  p.N = db->N;
  p.L = L;
  p.M = M;
  p.bins_per_chunk = lay.bpc;
  p.n_chunks = lay.n_chunks;
  p.n_qb = (int32_t)lay.n_qb;
  p.out_sign = db->metric == KNN_L2 ? -1.f : 1.f;
  p.zero_init = db->metric != KNN_L2;
  p.binV = binV;
  p.binA = binA;
  p.ldo = L;
  HIP_TRY(launch_fused(dt, ng, lay.ncb, p, s), "distance + bin-reduce kernel");
  if (bins_idx) HIP_TRY(launch_resolve(dt, binA, M, L, L, qbuf, db->tiles, ng, s), "resolve bin winners");
  const bool minimize = db->metric == KNN_L2;
  if (rerank_k <= 0) {
    HIP_TRY(launch_select(binV, binA, M, L, L, K, minimize, out_val, out_idx, K, s), "top-K select");
    HIP_TRY(launch_resolve(dt, out_idx, M, K, K, qbuf, db->tiles, ng, s), "resolve top-K rows");
    return KNN_OK;
  }
  float* cv = reinterpret_cast<float*>(ws + lay.cv);
  int32_t* ci = reinterpret_cast<int32_t*>(ws + lay.ci);
  HIP_TRY(launch_select(binV, binA, M, L, L, rerank_k, minimize, cv, ci, rerank_k, s),
          "top-K select (rerank candidates)");
  HIP_TRY(launch_resolve(dt, ci, M, rerank_k, rerank_k, qbuf, db->tiles, ng, s), "resolve rerank candidates");
  HIP_TRY(launch_rerank(ci, M, rerank_k, Q, q_dtype, db->X, db->in_dt, db->D, db->metric, db->orig_half_norm,
                        db->orig_rnorm, K, out_val, out_idx, s),
          "FP32 rerank");
  return KNN_OK;
}

extern "C" knn_status knn_db_search_workspace_size(const knn_db* db, int64_t M, int32_t K, int64_t L,
                                                   double recall_target, int64_t input_size_override,
                                                   int32_t rerank_k, int32_t with_bins, size_t* bytes) {
  g_last_error.clear();
  if (!db || !bytes) return fail(KNN_ERR_INVALID, "db and bytes must be non-NULL");
  L = resolve_bins(db->N, K, L, recall_target, input_size_override);
  if (L < 1) return fail(KNN_ERR_INVALID, "cannot derive L (K=%d, recall_target=%g)", K, recall_target);
  knn_status st = check_sizes(M, db->N, db->D, K, L);
  if (st != KNN_OK) return st;
  *bytes = search_layout(db, M, L, rerank_k, with_bins != 0).total;
  return KNN_OK;
}

extern "C" knn_status knn_db_search(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K,
                                    int64_t L, double recall_target, int64_t input_size_override, int32_t rerank_k,
                                    float* out_val, int32_t* out_idx, float* bins_val, int32_t* bins_idx,
                                    void* workspace, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  L = resolve_bins(db->N, K, L, recall_target, input_size_override);
  if (L < 1) return fail(KNN_ERR_INVALID, "cannot derive L (K=%d, recall_target=%g)", K, recall_target);
  knn_status st = check_search(db, Q, q_dtype, M, K, L, rerank_k, out_val, out_idx, bins_val, bins_idx);
  if (st != KNN_OK) return st;
  const size_t need = search_layout(db, M, L, rerank_k, bins_val != nullptr).total;
  if (ws_bytes < need)
    return fail(KNN_ERR_INVALID, "workspace too small (%zu < %zu bytes, see knn_db_search_workspace_size)",
                ws_bytes, need);
  if (need > 0 && (!workspace || reinterpret_cast<uintptr_t>(workspace) % 16 != 0))
    return fail(KNN_ERR_INVALID, "workspace must be a non-NULL, 16-byte aligned device pointer");
  return search_core(db, Q, q_dtype, M, K, L, rerank_k, out_val, out_idx, bins_val, bins_idx,
                     static_cast<unsigned char*>(workspace), (hipStream_t)stream);
}

extern "C" knn_status knn_search(const float* Q, int64_t M, const float* X, int64_t N, int32_t D, int32_t K,
                                 int64_t L, int32_t metric, float* out_val, int32_t* out_idx, void* stream) {
  g_last_error.clear();
  if (L <= 0) L = knn_bins_for_recall(K, 0.95, N);
  knn_status st = check_sizes(M, N, D, K, L);
  if (st != KNN_OK) return st;
  if (!valid_metric(metric)) return fail(KNN_ERR_INVALID, "bad metric %d", metric);
  if (!X || (M > 0 && (!Q || !out_val || !out_idx)))
    return fail(KNN_ERR_INVALID, "Q, X, out_val and out_idx must be non-NULL");
  if (M == 0) return KNN_OK;
  hipStream_t s = (hipStream_t)stream;
  knn_db db;
  db.in_dt = KNN_F32;
  db.compute = KNN_F32;
  db.metric = metric;
  db.D = D;
  db.dpad = dpad_for(D, KNN_F32);
  db.ng = groups_for(db.dpad, KNN_F32);
  db.N = N;
  db.n_tiles = ceil_div(N, kTileRows);
  db.X = X;
  // the plain form takes raw rows: it prepares X into a stream-ordered temporary from
  // the library's pool on every call, followed by the search's own workspace
  const size_t tiles_bytes = align_up((size_t)(db.n_tiles * tile_bytes(db.ng)));
  const size_t ws_bytes = search_layout(&db, M, L, 0, false).total;
  DevBuf tmp;
  HIP_TRY(tmp.alloc(tiles_bytes + ws_bytes, s), "hipMallocAsync (prepared rows and workspace)");
  db.tiles = static_cast<unsigned char*>(tmp.p);
  HIP_TRY(launch_prepare(X, KNN_F32, N, D, metric, KNN_F32, true, db.tiles, db.n_tiles, nullptr, nullptr, s),
          "database preparation");
  return search_core(&db, Q, KNN_F32, M, K, L, 0, out_val, out_idx, nullptr, nullptr,
                     static_cast<unsigned char*>(tmp.p) + tiles_bytes, s);
}

// --------------------------------------------------------------------------- allocation-free search
namespace {

// Fixed device scratch of knn_db_search_noalloc: the search's workspace for callers that
// cannot allocate.  Each device the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up per device (hipGetSymbolAddress) and only that is used.
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

knn_status scratch_of_current_device(unsigned char** out) {
  static std::mutex mu;
  static std::map<int, unsigned char*> addr;  // device -> address of its copy
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (scratch)");
    it = addr.emplace(dev, static_cast<unsigned char*>(p)).first;
  }
  *out = it->second;
  return KNN_OK;
}

}  // namespace

extern "C" size_t knn_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" knn_status knn_db_search_noalloc(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K,
                                            int64_t L, double recall_target, int64_t input_size_override,
                                            int32_t rerank_k, float* out_val, int32_t* out_idx, float* bins_val,
                                            int32_t* bins_idx, void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  L = resolve_bins(db->N, K, L, recall_target, input_size_override);
  if (L < 1) return fail(KNN_ERR_INVALID, "cannot derive L (K=%d, recall_target=%g)", K, recall_target);
  knn_status st = check_search(db, Q, q_dtype, M, K, L, rerank_k, out_val, out_idx, bins_val, bins_idx);
  if (st != KNN_OK) return st;
  const size_t need = search_layout(db, M, L, rerank_k, bins_val != nullptr).total;
  if (need > kScratchBytes)
    return fail(KNN_ERR_INVALID,
                "this search needs %zu bytes of scratch, more than the fixed %zu of knn_db_search_noalloc "
                "(fewer queries per call, fewer bins, a smaller rerank_k, or knn_db_search with a workspace)",
                need, kScratchBytes);
  if (M == 0) return KNN_OK;
  unsigned char* ws = nullptr;
  st = scratch_of_current_device(&ws);
  if (st != KNN_OK) return st;
  return search_core(db, Q, q_dtype, M, K, L, rerank_k, out_val, out_idx, bins_val, bins_idx, ws, (hipStream_t)stream);
}

// --------------------------------------------------------------------------- separate steps
static int64_t query_tiles_for(int64_t M) {
  // padded to the widest query block (kWaves * 32 * 2 queries) so any ncb can read it
  const int64_t QB = (int64_t)kWaves * 32 * 2;
  return ceil_div(std::max<int64_t>(M, 1), QB) * QB / kTileRows;
}

extern "C" size_t knn_query_buffer_bytes(const knn_db* db, int64_t M) {
  if (!db || M < 0) return 0;
  return (size_t)(query_tiles_for(M) * tile_bytes(db->ng));
}

extern "C" knn_status knn_query_prepare(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, void* qbuf,
                                        size_t qbuf_bytes, void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  if (M < 0) return fail(KNN_ERR_INVALID, "M must be >= 0");
  if (!valid_in(q_dtype)) return fail(KNN_ERR_INVALID, "q_dtype must be KNN_F32 or KNN_BF16");
  if (M > 0 && (!Q || !qbuf)) return fail(KNN_ERR_INVALID, "Q and qbuf must be non-NULL");
  if (qbuf_bytes < knn_query_buffer_bytes(db, M))
    return fail(KNN_ERR_INVALID, "qbuf too small (%zu < %zu bytes)", qbuf_bytes, knn_query_buffer_bytes(db, M));
  if (M == 0) return KNN_OK;
  HIP_TRY(launch_prepare(Q, q_dtype, M, db->D, db->metric, db->compute, false, (unsigned char*)qbuf,
                         query_tiles_for(M), nullptr, nullptr, (hipStream_t)stream),
          "query preparation");
  return KNN_OK;
}

extern "C" knn_status knn_partial_reduce(const knn_db* db, const void* qbuf, int64_t M, int64_t L, float* bins_val,
                                         int32_t* bins_idx, void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  if (M < 0) return fail(KNN_ERR_INVALID, "M must be >= 0");
  if (L < 1 || L > db->N) return fail(KNN_ERR_INVALID, "need 1 <= L <= N (L=%lld)", (long long)L);
  if (M > 0 && (!qbuf || !bins_val || !bins_idx)) return fail(KNN_ERR_INVALID, "NULL buffer");
  if (M == 0) return KNN_OK;
  const int ncb = pick_ncb(db->compute, db->ng, M);
  const int64_t QB = (int64_t)kWaves * 32 * ncb;
  const int64_t n_qb = ceil_div(M, QB);
  const int64_t bpc = pick_bins_per_chunk(db->N, L, n_qb, db->ng);
  FusedParams p{};
  p.db_tiles = db->tiles;
  p.q_tiles = (const unsigned char*)qbuf;
  p.N = db->N;
  p.L = L;
  p.M = M;
  p.bins_per_chunk = bpc;
  p.n_chunks = ceil_div(L, bpc);
  p.n_qb = (int32_t)n_qb;
  p.out_sign = db->metric == KNN_L2 ? -1.f : 1.f;
  p.zero_init = db->metric != KNN_L2;
  p.binV = bins_val;
  p.binA = bins_idx;
  p.ldo = L;
  HIP_TRY(launch_fused(db->compute, db->ng, ncb, p, (hipStream_t)stream), "distance + bin-reduce kernel");
  return KNN_OK;
}

extern "C" knn_status knn_resolve_rows(const knn_db* db, const void* qbuf, int64_t M, int64_t ncols, int32_t* idx,
                                       int64_t ld, void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  if (M < 0 || ncols < 0 || ld < ncols) return fail(KNN_ERR_INVALID, "bad sizes");
  if (M > 0 && ncols > 0 && (!qbuf || !idx)) return fail(KNN_ERR_INVALID, "NULL buffer");
  HIP_TRY(launch_resolve(db->compute, idx, M, ncols, ld, (const unsigned char*)qbuf, db->tiles, db->ng,
                         (hipStream_t)stream),
          "resolve rows");
  return KNN_OK;
}

// --------------------------------------------------------------------------- backward
extern "C" knn_status knn_backward(const float* g, const int32_t* idx, const void* Q, const void* X,
                                   int32_t in_dtype, int64_t M, int64_t N, int32_t D, int32_t K, int32_t metric,
                                   float* dQ, float* dX, void* stream) {
  g_last_error.clear();
  if (M < 0 || N < 1 || N > kMaxRows || D < 1 || K < 1)
    return fail(KNN_ERR_INVALID, "bad sizes (M=%lld N=%lld D=%d K=%d)", (long long)M, (long long)N, D, K);
  if (D > kMaxDpad) return fail(KNN_ERR_UNSUPPORTED, "D must be <= %d", kMaxDpad);
  if (!valid_in(in_dtype)) return fail(KNN_ERR_INVALID, "in_dtype must be KNN_F32 or KNN_BF16");
  if (!valid_metric(metric)) return fail(KNN_ERR_INVALID, "bad metric %d", metric);
  if (M > 0 && (!g || !idx || !Q || !X || !dQ)) return fail(KNN_ERR_INVALID, "g, idx, Q, X and dQ must be non-NULL");
  HIP_TRY(launch_backward(g, idx, Q, X, in_dtype, M, N, D, K, metric, dQ, dX, (hipStream_t)stream), "backward");
  return KNN_OK;
}

// --------------------------------------------------------------------------- approx_max_k on scores
extern "C" int64_t knn_approx_bins(int64_t n, int32_t K, double recall_target, int64_t input_size_override) {
  if (n < 1 || K < 1 || K > n) return -1;
  const int64_t n_eval = input_size_override > 0 ? input_size_override : n;
  const int64_t L_eval = knn_bins_for_recall(K, recall_target, n_eval);
  if (L_eval < 1) return -1;
  int64_t L = L_eval;
  if (input_size_override > 0) {
    // the same bin density as the L_eval bins of the n_eval-long slice this one is part of
    L = (int64_t)std::ceil((double)L_eval * (double)n / (double)n_eval);
  }
  return std::min<int64_t>(std::max<int64_t>(L, K), n);
}

namespace {

// Checks the op's arguments and resolves L; on success B (slices), n (slice length)
// and L are set and the workspace need (bins of every slice when aggregating) is returned
// in *ws.
knn_status approx_args(int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int32_t& reduction_dim, int32_t K,
                       double recall_target, int64_t input_size_override, int64_t& L, int32_t minimize,
                       int32_t aggregate_to_topk, int64_t& B, int64_t& n, size_t* ws) {
  if (dtype != KNN_F32 && dtype != KNN_BF16) return fail(KNN_ERR_INVALID, "dtype must be KNN_F32 or KNN_BF16");
  if (rows < 0 || cols < 0) return fail(KNN_ERR_INVALID, "rows and cols must be >= 0");
  if (ld < cols || ld < 1) return fail(KNN_ERR_INVALID, "need ld >= max(cols, 1) (ld=%lld)", (long long)ld);
  if (reduction_dim == -1) reduction_dim = 1;
  if (reduction_dim != 0 && reduction_dim != 1) return fail(KNN_ERR_INVALID, "reduction_dim must be 0, 1 or -1");
  if (minimize != 0 && minimize != 1) return fail(KNN_ERR_INVALID, "minimize must be 0 or 1");
  if (aggregate_to_topk != 0 && aggregate_to_topk != 1) return fail(KNN_ERR_INVALID, "aggregate_to_topk must be 0 or 1");
  n = reduction_dim == 1 ? cols : rows;
  B = reduction_dim == 1 ? rows : cols;
  if (n < 1 || n > kMaxRows)
    return fail(KNN_ERR_INVALID, "the reduced dimension must have 1 .. 2^31 - 64 entries (got %lld)", (long long)n);
  if (K < 1 || K > n) return fail(KNN_ERR_INVALID, "need 1 <= K <= reduced size (K=%d, n=%lld)", K, (long long)n);
  if (aggregate_to_topk && K > 1024) return fail(KNN_ERR_INVALID, "K must be <= 1024 (got %d)", K);
  if (L <= 0) {
    if (!(recall_target > 0.0 && recall_target < 1.0))
      return fail(KNN_ERR_INVALID, "recall_target must be in (0, 1)");
    L = knn_approx_bins(n, K, recall_target, input_size_override);
  }
  if (L < K || L > n)
    return fail(KNN_ERR_INVALID, "need K <= L <= reduced size (K=%d, L=%lld, n=%lld)", K, (long long)L, (long long)n);
  *ws = (aggregate_to_topk && B > 0) ? align_up(sizeof(float) * (size_t)(B * L)) + align_up(sizeof(int32_t) * (size_t)(B * L))
                                     : 0;
  return KNN_OK;
}

}  // namespace

extern "C" knn_status knn_approx_workspace_size(int32_t dtype, int64_t rows, int64_t cols, int64_t ld,
                                                int32_t reduction_dim, int32_t K, double recall_target,
                                                int64_t input_size_override, int64_t L, int32_t minimize,
                                                int32_t aggregate_to_topk, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(KNN_ERR_INVALID, "bytes is NULL");
  int64_t B = 0, n = 0;
  return approx_args(dtype, rows, cols, ld, reduction_dim, K, recall_target, input_size_override, L, minimize,
                     aggregate_to_topk, B, n, bytes);
}

extern "C" knn_status knn_approx_top_k(const void* scores, int32_t dtype, int64_t rows, int64_t cols, int64_t ld,
                                       int32_t reduction_dim, int32_t K, double recall_target,
                                       int64_t input_size_override, int64_t L, int32_t minimize,
                                       int32_t aggregate_to_topk, float* out_val, int32_t* out_idx, void* workspace,
                                       size_t ws_bytes, void* stream) {
  g_last_error.clear();
  int64_t B = 0, n = 0;
  size_t need = 0;
  knn_status st = approx_args(dtype, rows, cols, ld, reduction_dim, K, recall_target, input_size_override, L,
                              minimize, aggregate_to_topk, B, n, &need);
  if (st != KNN_OK) return st;
  if (B > 0 && (!scores || !out_val || !out_idx)) return fail(KNN_ERR_INVALID, "scores and outputs must be non-NULL");
  const size_t esz = dtype == KNN_F32 ? 4 : 2;
  if (reinterpret_cast<uintptr_t>(scores) % esz != 0) return fail(KNN_ERR_INVALID, "scores must be %zu-byte aligned", esz);
  if (ws_bytes < need)
    return fail(KNN_ERR_INVALID, "workspace too small (%zu < %zu bytes, see knn_approx_workspace_size)", ws_bytes,
                need);
  if (need > 0 && (!workspace || reinterpret_cast<uintptr_t>(workspace) % 16 != 0))
    return fail(KNN_ERR_INVALID, "workspace must be a non-NULL, 16-byte aligned device pointer");
  if (B == 0) return KNN_OK;
  hipStream_t s = (hipStream_t)stream;
  const int dt = dtype == KNN_F32 ? DT_F32 : DT_BF16;
  if (!aggregate_to_topk) {
    HIP_TRY(launch_approx_bins(scores, dt, rows, cols, ld, reduction_dim, L, minimize != 0, out_val, out_idx, s),
            "approx bins");
    return KNN_OK;
  }
  float* V = static_cast<float*>(workspace);
  int32_t* A = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(workspace) + align_up(sizeof(float) * (size_t)(B * L)));
  HIP_TRY(launch_approx_bins(scores, dt, rows, cols, ld, reduction_dim, L, minimize != 0, V, A, s), "approx bins");
  if (reduction_dim == 1)  // bins B x L, results B x K
    HIP_TRY(launch_select(V, A, B, L, L, K, minimize != 0, out_val, out_idx, K, s), "top-K");
  else  // bins L x B (bin-major), results K x B
    HIP_TRY(launch_select(V, A, B, L, 1, K, minimize != 0, out_val, out_idx, 1, s, B, B), "top-K");
  return KNN_OK;
}

// --------------------------------------------------------------------------- batched plan
namespace {

constexpr int kPlanBlocksPerXcd = 64;  // 2 resident workgroups on each of an XCD's 32 CUs
constexpr int kPlanBlocks = 8 * kPlanBlocksPerXcd;

void set_group_shape(GroupPlan& g) {
  const int64_t QB = (int64_t)kWaves * 32 * g.ncb;
  g.n_qb = ceil_div(std::max<int64_t>(g.M, 1), QB);
  g.q_tiles_n = g.n_qb * QB / kTileRows;
  g.n_chunks = ceil_div(g.L, g.bins_per_chunk);
}

// With knn_plan_set_own_launches: a group with enough (query block, chunk) items to
// fill the GPU for several rounds runs as a launch of the distance kernel specialised
// for its depth (e.g. three waves per SIMD at depth 128, where the persistent kernel,
// which holds every depth's code, runs two).  The others share the persistent launch,
// which balances them against one another.
void set_own_launch(const knn_plan* p, GroupPlan& g) {
  g.own = p->own_launch_items > 0 && g.M > 0 && g.n_chunks * g.n_qb >= p->own_launch_items;
}

// the autotuner's candidates for one group: L at or above the L2-resident choice (a bin
// that does not fit the 2 MiB an XCD's workgroups stream through its L2 is re-fetched
// by every query block), ncb in {1, 2}, two work-item sizes
std::vector<GroupPlan> tune_candidates(const knn_plan* p, const GroupPlan& g) {
  std::vector<GroupPlan> out;
  const knn_db* db = p->dbs[g.db];
  const int64_t N = db->N;
  const int64_t Lfit = std::min<int64_t>(N, std::max(g.L_min, bins_for_l2(N, db->ng)));
  for (int64_t Lc : {Lfit, std::min<int64_t>(N, 2 * Lfit)}) {
    for (int ncb : {1, 2}) {
      if (!fused_supported(p->compute, db->ng, ncb)) continue;
      const int64_t QB = (int64_t)kWaves * 32 * ncb;
      const int64_t nqb = ceil_div(std::max<int64_t>(g.M, 1), QB);
      for (int64_t target : {int64_t(1024), int64_t(4096)}) {
        GroupPlan c = g;
        c.L = Lc;
        c.ncb = ncb;
        c.bins_per_chunk = pick_bins_per_chunk(N, Lc, nqb, db->ng, target);
        set_group_shape(c);
        bool dup = false;
        for (const auto& o : out) dup |= (o.L == c.L && o.ncb == c.ncb && o.bins_per_chunk == c.bins_per_chunk);
        if (!dup) out.push_back(c);
      }
    }
  }
  return out;
}

// Device memory of the plan for its current choices, as offsets into the workspace:
// per group the prepared queries and the M x L bins, then the descriptors, then the
// autotuner's top-K output.  With `items_bound` >= 0 the work list is sized for that
// many items instead of the current ones.
struct PlanLayout {
  std::vector<size_t> q, bv, ba;
  size_t segs = 0, gds = 0, items = 0, claim = 0, sel = 0, tv = 0, ti = 0, total = 0;
};

int64_t count_sel_rows(const knn_plan* p) {
  int64_t n = 0;
  for (const auto& b : p->batches) n += b.M;
  return n;
}

PlanLayout plan_layout(const knn_plan* p, const std::vector<GroupPlan>& groups, int64_t n_items) {
  PlanLayout l;
  size_t off = 0;
  int64_t tune_rows = 0;
  for (const auto& g : groups) {
    const knn_db* db = p->dbs[g.db];
    l.q.push_back(off);
    off += align_up((size_t)(g.q_tiles_n * tile_bytes(db->ng)));
    l.bv.push_back(off);
    off += align_up(sizeof(float) * (size_t)std::max<int64_t>(1, g.M * g.L));
    l.ba.push_back(off);
    off += align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(1, g.M * g.L));
    tune_rows = std::max<int64_t>(tune_rows, g.M * g.K_max);
  }
  l.segs = off;
  off += align_up(sizeof(QSeg) * (p->batches.size() + groups.size() + 1));
  l.gds = off;
  off += align_up(sizeof(GroupDesc) * (groups.size() + 1));
  l.items = off;
  off += align_up(sizeof(WorkItem) * (size_t)std::max<int64_t>(1, n_items));
  l.claim = off;
  off += align_up(sizeof(unsigned) * 8);
  l.sel = off;
  off += align_up(sizeof(SelRow) * (size_t)std::max<int64_t>(1, count_sel_rows(p)));
  l.tv = off;
  off += align_up(sizeof(float) * (size_t)std::max<int64_t>(1, tune_rows));
  l.ti = off;
  off += align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(1, tune_rows));
  l.total = off;
  return l;
}

// work list: chunks dealt round-robin to the 8 XCDs; the items of one chunk (all its
// query blocks) are consecutive in that XCD's list, so the persistent workgroups of one
// XCD, which take the list in order, share a chunk's tiles through its L2.  The 8 lists
// are stored one after another, each padded to the longest.
std::vector<WorkItem> build_items(const std::vector<GroupPlan>& groups) {
  std::vector<std::vector<WorkItem>> per_xcd(8);
  int64_t chunk_seq = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const GroupPlan& g = groups[gi];
    if (g.M == 0 || g.own) continue;  // own launch (run_plan)
    for (int64_t c = 0; c < g.n_chunks; ++c, ++chunk_seq) {
      auto& lst = per_xcd[chunk_seq % 8];
      for (int64_t qb = 0; qb < g.n_qb; ++qb) {
        WorkItem it{};
        it.grp = (int32_t)gi;
        it.qb = (int32_t)qb;
        it.b0 = c * g.bins_per_chunk;
        it.b1 = std::min(g.L, it.b0 + g.bins_per_chunk);
        lst.push_back(it);
      }
    }
  }
  size_t len = 0;
  for (auto& l : per_xcd) len = std::max(len, l.size());
  WorkItem pad{};
  pad.grp = -1;
  std::vector<WorkItem> items(8 * len, pad);
  for (int x = 0; x < 8; ++x) std::copy(per_xcd[x].begin(), per_xcd[x].end(), items.begin() + (size_t)x * len);
  return items;
}

// Upper bound of the work list over every choice the autotuner may try: per XCD at most
// ceil(chunks / 8) + 1 chunks of each group, each with its query blocks.
int64_t items_bound(const knn_plan* p) {
  int64_t per_xcd = 0;
  for (const auto& g : p->groups) {
    if (g.M == 0) continue;
    int64_t worst = (ceil_div(g.n_chunks, 8) + 1) * g.n_qb;
    if (g.tune)
      for (const auto& c : tune_candidates(p, g)) worst = std::max(worst, (ceil_div(c.n_chunks, 8) + 1) * c.n_qb);
    per_xcd += worst;
  }
  return ceil_div(std::max<int64_t>(per_xcd, 1), kPlanBlocksPerXcd) * kPlanBlocks;
}

size_t plan_bound_bytes(const knn_plan* p) {
  // every group at its largest candidate buffers, the work list at its bound
  std::vector<GroupPlan> big = p->groups;
  for (auto& g : big) {
    if (!g.tune) continue;
    for (const auto& c : tune_candidates(p, g)) {
      if (c.M * c.L > g.M * g.L) g.L = c.L;
      if (c.q_tiles_n > g.q_tiles_n) g.q_tiles_n = c.q_tiles_n;
    }
  }
  return plan_layout(p, big, items_bound(p)).total;
}

// Lay out the plan's current choices in the workspace and upload its descriptors.
knn_status bind_plan(knn_plan* p, unsigned char* ws, hipStream_t s) {
  for (auto& g : p->groups) {
    set_group_shape(g);
    set_own_launch(p, g);
  }
  p->items = build_items(p->groups);
  const PlanLayout lay = plan_layout(p, p->groups, items_bound(p));
  p->segs.clear();
  p->gds.clear();
  p->sel.clear();
  int64_t first = 0;
  p->max_ng = 0;
  p->lds_bytes = 0;
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    GroupPlan& g = p->groups[gi];
    const knn_db* db = p->dbs[g.db];
    g.q_tiles = ws + lay.q[gi];
    g.binV = reinterpret_cast<float*>(ws + lay.bv[gi]);
    g.binA = reinterpret_cast<int32_t*>(ws + lay.ba[gi]);
    p->max_ng = std::max(p->max_ng, db->ng);
    p->lds_bytes = std::max(p->lds_bytes, fused_lds_bytes(p->compute, db->ng, g.ncb));
    // query segments: the batches of this group in order, then padding rows
    int64_t row = 0;
    for (const auto& b : p->batches) {
      if (b.db != g.db || b.M == 0) continue;
      QSeg q{};
      q.src = b.Q;
      q.first = first;
      q.rows = b.M;
      q.dst_row0 = row;
      q.D = db->D;
      q.ng = db->ng;
      q.metric = db->metric;
      q.tiles = g.q_tiles;
      p->segs.push_back(q);
      for (int64_t r = 0; r < b.M; ++r) {
        SelRow sr{};
        sr.V = g.binV + (row + r) * g.L;
        sr.A = g.binA + (row + r) * g.L;
        sr.n = g.L;
        sr.K = b.K;
        sr.minimize = db->metric == KNN_L2;
        sr.out_val = b.out_val + r * b.K;
        sr.out_idx = b.out_idx + r * b.K;
        sr.q_tiles = g.q_tiles;
        sr.db_tiles = db->tiles;
        sr.q_row = row + r;
        sr.ng = db->ng;
        p->sel.push_back(sr);
      }
      first += b.M;
      row += b.M;
    }
    const int64_t padded = g.q_tiles_n * kTileRows;
    if (padded > row) {
      QSeg q{};
      q.src = nullptr;
      q.first = first;
      q.rows = 0;
      q.dst_row0 = row;
      q.D = db->D;
      q.ng = db->ng;
      q.metric = db->metric;
      q.tiles = g.q_tiles;
      p->segs.push_back(q);
      first += padded - row;
    }
    GroupDesc gd{};
    gd.db_tiles = db->tiles;
    gd.q_tiles = g.q_tiles;
    gd.N = db->N;
    gd.L = g.L;
    gd.M = g.M;
    gd.out_sign = db->metric == KNN_L2 ? -1.f : 1.f;
    gd.binV = g.binV;
    gd.binA = g.binA;
    gd.ldo = g.L;
    gd.ng = db->ng;
    gd.ncb = g.ncb;
    gd.zero_init = db->metric != KNN_L2;
    p->gds.push_back(gd);
  }
  p->total_q_rows = first;
  p->n_segs = (int)p->segs.size();
  p->n_sel_rows = (int64_t)p->sel.size();
  p->n_blocks = kPlanBlocks;
  p->n_items = (int64_t)p->items.size();
  p->d_segs = reinterpret_cast<QSeg*>(ws + lay.segs);
  p->d_groups = reinterpret_cast<GroupDesc*>(ws + lay.gds);
  p->d_items = reinterpret_cast<WorkItem*>(ws + lay.items);
  p->d_claim = reinterpret_cast<unsigned*>(ws + lay.claim);
  p->d_sel = reinterpret_cast<SelRow*>(ws + lay.sel);
  p->tune_val = reinterpret_cast<float*>(ws + lay.tv);
  p->tune_idx = reinterpret_cast<int32_t*>(ws + lay.ti);
  HIP_TRY(hipMemcpyAsync(p->d_segs, p->segs.data(), sizeof(QSeg) * p->segs.size(), hipMemcpyHostToDevice, s),
          "upload");
  HIP_TRY(hipMemcpyAsync(p->d_groups, p->gds.data(), sizeof(GroupDesc) * p->gds.size(), hipMemcpyHostToDevice, s),
          "upload");
  HIP_TRY(hipMemcpyAsync(p->d_items, p->items.data(), sizeof(WorkItem) * p->items.size(), hipMemcpyHostToDevice, s),
          "upload");
  if (!p->sel.empty())
    HIP_TRY(hipMemcpyAsync(p->d_sel, p->sel.data(), sizeof(SelRow) * p->sel.size(), hipMemcpyHostToDevice, s),
            "upload");
  // the host descriptors are rewritten by the next bind: wait for the copies
  HIP_TRY(hipStreamSynchronize(s), "sync");
  return KNN_OK;
}

// the distance launch of one group on its own (its queries prepared by the plan)
FusedParams group_params(const knn_plan* p, const GroupPlan& g) {
  const knn_db* db = p->dbs[g.db];
  FusedParams fp{};
  fp.db_tiles = db->tiles;
  fp.q_tiles = g.q_tiles;
  fp.N = db->N;
  fp.L = g.L;
  fp.M = g.M;
  fp.bins_per_chunk = g.bins_per_chunk;
  fp.n_chunks = g.n_chunks;
  fp.n_qb = (int32_t)g.n_qb;
  fp.out_sign = db->metric == KNN_L2 ? -1.f : 1.f;
  fp.zero_init = db->metric != KNN_L2;
  fp.binV = g.binV;
  fp.binA = g.binA;
  fp.ldo = g.L;
  return fp;
}

knn_status run_plan(knn_plan* p, hipStream_t s) {
  HIP_TRY(launch_prepare_segments(p->d_segs, p->n_segs, p->total_q_rows, p->q_dtype, p->compute, s),
          "batched query preparation");
  for (const auto& g : p->groups)
    if (g.own)
      HIP_TRY(launch_fused(p->dbs[g.db]->compute, p->dbs[g.db]->ng, g.ncb, group_params(p, g), s),
              "distance + bin-reduce kernel (one database group)");
  HIP_TRY(launch_fused_persistent(p->compute, p->d_groups, p->d_items, p->n_items, p->d_claim, p->n_blocks,
                                  p->lds_bytes, s),
          "persistent distance + bin-reduce kernel");
  HIP_TRY(launch_select_rows(p->d_sel, p->n_sel_rows, p->max_K, s), "batched top-K select");
  HIP_TRY(launch_resolve_rows(p->compute, p->d_sel, p->n_sel_rows, s), "batched resolve");
  return KNN_OK;
}

// time one group alone with its current (ncb, L, bins_per_chunk): non-persistent
// distance launch + top-K, best of 3, the queries prepared by the plan's own launch
double time_group(knn_plan* p, size_t gi, hipStream_t s) {
  const GroupPlan& g = p->groups[gi];
  const knn_db* db = p->dbs[g.db];
  const FusedParams fp = group_params(p, g);
  hipEvent_t a, b;
  double best = 1e30;
  if (hipEventCreate(&a) != hipSuccess) return best;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return best;
  }
  if (launch_prepare_segments(p->d_segs, p->n_segs, p->total_q_rows, p->q_dtype, p->compute, s) == hipSuccess &&
      launch_fused(db->compute, db->ng, g.ncb, fp, s) == hipSuccess) {  // warm-up
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(a, s);
      (void)launch_fused(db->compute, db->ng, g.ncb, fp, s);
      (void)launch_select(g.binV, g.binA, g.M, g.L, g.L, g.K_max, false, p->tune_val, p->tune_idx, g.K_max, s);
      (void)hipEventRecord(b, s);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      best = std::min(best, (double)ms);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(s);
  return best;
}

std::string tune_key(const knn_plan* p, const GroupPlan& g) {
  const knn_db* db = p->dbs[g.db];
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  std::ostringstream o;
  o << prop.gcnArchName << "|dt" << db->compute << "|m" << db->metric << "|N" << db->N << "|D" << db->D << "|M"
    << g.M << "|K" << g.K_max << "|Lmin" << g.L_min;
  return o.str();
}

// tiny JSON cache: {"key": [L, ncb, bins_per_chunk], ...}
std::map<std::string, std::vector<int64_t>> read_cache(const std::string& path) {
  std::map<std::string, std::vector<int64_t>> m;
  if (path.empty()) return m;
  std::ifstream f(path);
  if (!f) return m;
  std::string all((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  size_t pos = 0;
  while (true) {
    size_t k0 = all.find('"', pos);
    if (k0 == std::string::npos) break;
    size_t k1 = all.find('"', k0 + 1);
    if (k1 == std::string::npos) break;
    size_t b0 = all.find('[', k1), b1 = all.find(']', b0);
    if (b0 == std::string::npos || b1 == std::string::npos) break;
    std::vector<int64_t> v;
    std::stringstream ss(all.substr(b0 + 1, b1 - b0 - 1));
    std::string tok;
    while (std::getline(ss, tok, ',')) v.push_back(std::atoll(tok.c_str()));
    m[all.substr(k0 + 1, k1 - k0 - 1)] = v;
    pos = b1 + 1;
  }
  return m;
}

void write_cache(const std::string& path, const std::map<std::string, std::vector<int64_t>>& m) {
  if (path.empty()) return;
  std::ofstream f(path);
  if (!f) return;
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : m) {
    f << "  \"" << kv.first << "\": [";
    for (size_t j = 0; j < kv.second.size(); ++j) f << (j ? ", " : "") << kv.second[j];
    f << "]" << (++i < m.size() ? "," : "") << "\n";
  }
  f << "}\n";
}

// A cached choice is used only if it is one the plan could have made: L between the
// recall bound (and K) and N, a kernel instance that exists, whole bins per item.
bool cached_choice_valid(const knn_plan* p, const GroupPlan& g, const std::vector<int64_t>& v) {
  if (v.size() != 3) return false;
  const knn_db* db = p->dbs[g.db];
  const int64_t L = v[0], ncb = v[1], bpc = v[2];
  if (L < std::max<int64_t>(g.L_min, g.K_max) || L > db->N) return false;
  if (ncb != 1 && ncb != 2) return false;
  if (!fused_supported(p->compute, db->ng, (int)ncb)) return false;
  return bpc >= 1 && bpc <= L;
}

}  // namespace

extern "C" knn_status knn_plan_create(knn_db* const* dbs, int32_t ndb, const knn_batch* batches, int32_t nb,
                                      int32_t q_dtype, double recall_target, int32_t tune, const char* cache_path,
                                      knn_plan** out) {
  g_last_error.clear();
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!dbs || ndb < 1) return fail(KNN_ERR_INVALID, "need at least one database");
  if (!batches || nb < 1) return fail(KNN_ERR_INVALID, "need at least one batch");
  if (!valid_in(q_dtype)) return fail(KNN_ERR_INVALID, "q_dtype must be KNN_F32 or KNN_BF16");
  if (!(recall_target > 0.0 && recall_target < 1.0)) return fail(KNN_ERR_INVALID, "recall_target must be in (0, 1)");
  for (int i = 0; i < ndb; ++i)
    if (!dbs[i]) return fail(KNN_ERR_INVALID, "database %d is NULL", i);
  const int compute = dbs[0]->compute;
  for (int i = 0; i < ndb; ++i) {
    if (dbs[i]->compute != compute) return fail(KNN_ERR_UNSUPPORTED, "all databases must share one compute type");
    if (compute != KNN_BF16) return fail(KNN_ERR_UNSUPPORTED, "the batched kernel is built for BF16 databases");
    const int ng = dbs[i]->ng;
    if (!(ng == 4 || ng == 6 || ng == 8 || ng == 16))
      return fail(KNN_ERR_UNSUPPORTED, "batched search supports padded depths 64, 96, 128 and 256 (database %d)", i);
  }
  for (int b = 0; b < nb; ++b) {
    const knn_batch& x = batches[b];
    if (x.db < 0 || x.db >= ndb) return fail(KNN_ERR_INVALID, "batch %d: bad database index %d", b, x.db);
    if (x.M < 0) return fail(KNN_ERR_INVALID, "batch %d: M < 0", b);
    if (x.K < 1 || x.K > 1024 || x.K > dbs[x.db]->N) return fail(KNN_ERR_INVALID, "batch %d: bad K %d", b, x.K);
    if (x.M > 0 && (!x.Q || !x.out_val || !x.out_idx)) return fail(KNN_ERR_INVALID, "batch %d: NULL pointer", b);
  }
  auto* p = new (std::nothrow) knn_plan();
  if (!p) return fail(KNN_ERR_OOM, "host allocation");
  p->dbs.assign(dbs, dbs + ndb);
  p->batches.assign(batches, batches + nb);
  p->q_dtype = q_dtype;
  p->compute = compute;
  if (cache_path) p->cache_path = cache_path;
  for (int d = 0; d < ndb; ++d) {
    GroupPlan g;
    g.db = d;
    for (const auto& b : p->batches)
      if (b.db == d) {
        g.M += b.M;
        g.K_max = std::max(g.K_max, b.K);
      }
    p->max_K = std::max(p->max_K, g.K_max);
    const int64_t N = dbs[d]->N;
    g.L = std::max<int64_t>(knn_bins_for_recall(g.K_max, recall_target, N), g.K_max);
    g.L_min = g.L;
    g.L = std::min<int64_t>(N, std::max(g.L, bins_for_l2(N, dbs[d]->ng)));
    g.ncb = g.M > 128 ? 2 : 1;
    const int64_t QB = (int64_t)kWaves * 32 * g.ncb;
    g.bins_per_chunk = pick_bins_per_chunk(N, g.L, ceil_div(std::max<int64_t>(g.M, 1), QB), dbs[d]->ng, 4096);
    set_group_shape(g);
    p->groups.push_back(g);
  }
  if (tune) {
    const auto cache = read_cache(p->cache_path);
    for (auto& g : p->groups) {
      if (g.M == 0) continue;
      auto it = cache.find(tune_key(p, g));
      if (it != cache.end() && cached_choice_valid(p, g, it->second)) {
        g.L = it->second[0];
        g.ncb = (int32_t)it->second[1];
        g.bins_per_chunk = it->second[2];
        set_group_shape(g);
      } else {
        g.tune = true;  // timed in knn_plan_setup
      }
    }
  }
  *out = p;
  return KNN_OK;
}

extern "C" knn_status knn_plan_workspace_size(const knn_plan* plan, size_t* bytes) {
  g_last_error.clear();
  if (!plan || !bytes) return fail(KNN_ERR_INVALID, "plan and bytes must be non-NULL");
  *bytes = plan_bound_bytes(plan);
  return KNN_OK;
}

extern "C" knn_status knn_plan_setup(knn_plan* p, void* workspace, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(KNN_ERR_INVALID, "plan is NULL");
  const size_t need = plan_bound_bytes(p);
  if (ws_bytes < need)
    return fail(KNN_ERR_INVALID, "workspace too small (%zu < %zu bytes, see knn_plan_workspace_size)", ws_bytes, need);
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 16 != 0)
    return fail(KNN_ERR_INVALID, "workspace must be a non-NULL, 16-byte aligned device pointer");
  hipStream_t s = (hipStream_t)stream;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  p->bound = false;
  bool tuned = false;
  auto cache = read_cache(p->cache_path);
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    if (!p->groups[gi].tune) continue;
    const GroupPlan start = p->groups[gi];
    double best = 1e30;
    GroupPlan bestg = start;
    for (const auto& c : tune_candidates(p, start)) {
      p->groups[gi] = c;
      if (bind_plan(p, ws, s) != KNN_OK) continue;
      const double ms = time_group(p, gi, s);
      if (ms < best) {
        best = ms;
        bestg = c;
      }
    }
    bestg.tune = false;
    p->groups[gi] = bestg;
    cache[tune_key(p, bestg)] = {bestg.L, bestg.ncb, bestg.bins_per_chunk};
    tuned = true;
  }
  if (tuned) write_cache(p->cache_path, cache);
  knn_status st = bind_plan(p, ws, s);
  if (st != KNN_OK) return st;
  p->bound = true;
  return KNN_OK;
}

extern "C" knn_status knn_search_batched(knn_plan* plan, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(KNN_ERR_INVALID, "plan is NULL");
  if (!plan->bound) return fail(KNN_ERR_INVALID, "plan has no workspace: call knn_plan_setup first");
  return run_plan(plan, (hipStream_t)stream);
}

extern "C" knn_status knn_plan_set_own_launches(knn_plan* plan, int64_t min_items) {
  g_last_error.clear();
  if (!plan) return fail(KNN_ERR_INVALID, "plan is NULL");
  if (min_items < 0) return fail(KNN_ERR_INVALID, "min_items must be >= 0 (got %lld)", (long long)min_items);
  plan->own_launch_items = min_items;
  plan->bound = false;  // the work list changes: knn_plan_setup again
  return KNN_OK;
}

extern "C" knn_status knn_plan_info(const knn_plan* plan, int64_t* L, int32_t* qblock, int64_t* chunk_rows) {
  g_last_error.clear();
  if (!plan) return fail(KNN_ERR_INVALID, "plan is NULL");
  for (size_t i = 0; i < plan->groups.size(); ++i) {
    const GroupPlan& g = plan->groups[i];
    if (L) L[i] = g.L;
    if (qblock) qblock[i] = kWaves * 32 * g.ncb;
    if (chunk_rows) chunk_rows[i] = (int64_t)((double)plan->dbs[g.db]->N / (double)g.L * (double)g.bins_per_chunk);
  }
  return KNN_OK;
}

extern "C" knn_status knn_plan_destroy(knn_plan* plan) {
  delete plan;  // its workspace is the caller's memory
  return KNN_OK;
}
