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
struct knn_db {
  int32_t in_dt, compute, metric, D, dpad, ng;
  int64_t N, n_tiles;
  unsigned char* tiles = nullptr;
  float* orig_half_norm = nullptr;  // L2: |x|^2/2 of the original rows (rerank)
  float* orig_rnorm = nullptr;      // cosine: 1/|x| of the original rows (rerank)
  const void* X = nullptr;          // caller's rows (not owned)
};

struct GroupPlan {
  int32_t db;
  int64_t M = 0, L = 0, L_min = 0, bins_per_chunk = 0, n_qb = 0, n_chunks = 0, q_tiles_n = 0;
  int32_t ncb = 1, K_max = 1;
  unsigned char* q_tiles = nullptr;
  float* binV = nullptr;
  int32_t* binA = nullptr;
};

struct knn_plan {
  std::vector<knn_db*> dbs;
  std::vector<knn_batch> batches;
  std::vector<GroupPlan> groups;
  int32_t q_dtype = KNN_F32, compute = KNN_BF16;
  int64_t total_q_rows = 0, n_items = 0, n_sel_rows = 0;
  int n_blocks = 0, max_ng = 0, n_segs = 0, max_K = 1, lds_bytes = 0;
  QSeg* d_segs = nullptr;
  GroupDesc* d_groups = nullptr;
  WorkItem* d_items = nullptr;
  SelRow* d_sel = nullptr;
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
extern "C" knn_status knn_db_create(const void* X, int32_t in_dtype, int64_t N, int32_t D, int32_t metric,
                                    int32_t compute, void* stream, knn_db** out) {
  g_last_error.clear();
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  if (!X) return fail(KNN_ERR_INVALID, "X is NULL");
  if (!valid_in(in_dtype)) return fail(KNN_ERR_INVALID, "in_dtype must be KNN_F32 or KNN_BF16");
  if (!valid_compute(compute)) return fail(KNN_ERR_INVALID, "bad compute dtype %d", compute);
  if (!valid_metric(metric)) return fail(KNN_ERR_INVALID, "bad metric %d", metric);
  if (N < 1 || N > kMaxRows) return fail(KNN_ERR_INVALID, "N must be in [1, 2^31 - 64]");
  if (D < 1) return fail(KNN_ERR_INVALID, "D must be >= 1");
  if (D > kMaxDpad) return fail(KNN_ERR_UNSUPPORTED, "D must be <= %d", kMaxDpad);
  hipStream_t s = (hipStream_t)stream;
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
  hipError_t e = hipMalloc(&db->tiles, (size_t)(db->n_tiles * tile_bytes(db->ng)));
  if (e == hipSuccess && metric == KNN_L2) e = hipMalloc(&db->orig_half_norm, sizeof(float) * (size_t)N);
  if (e == hipSuccess && metric == KNN_COSINE) e = hipMalloc(&db->orig_rnorm, sizeof(float) * (size_t)N);
  if (e != hipSuccess) {
    knn_db_destroy(db);
    return fail(KNN_ERR_OOM, "hipMalloc for the prepared database: %s", hipGetErrorString(e));
  }
  e = launch_prepare(X, in_dtype, N, D, metric, compute, true, db->tiles, db->n_tiles, db->orig_half_norm,
                     db->orig_rnorm, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    knn_db_destroy(db);
    return hip_fail(e, "database preparation");
  }
  *out = db;
  return KNN_OK;
}

extern "C" knn_status knn_db_destroy(knn_db* db) {
  if (!db) return KNN_OK;
  if (db->tiles) (void)hipFree(db->tiles);
  if (db->orig_half_norm) (void)hipFree(db->orig_half_norm);
  if (db->orig_rnorm) (void)hipFree(db->orig_rnorm);
  delete db;
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
static knn_status search_core(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K, int64_t L,
                              int32_t rerank_k, float* out_val, int32_t* out_idx, float* bins_val,
                              int32_t* bins_idx, hipStream_t s) {
  if (M == 0) return KNN_OK;
  const int dt = db->compute, ng = db->ng;
  const int ncb = pick_ncb(dt, ng, M);
  const int64_t QB = (int64_t)kWaves * 32 * ncb;
  const int64_t n_qb = ceil_div(M, QB);
  const int64_t q_tiles_n = n_qb * QB / kTileRows;
  const int64_t bpc = pick_bins_per_chunk(db->N, L, n_qb, db->ng);
  const int64_t n_chunks = ceil_div(L, bpc);

  DevBuf qbuf, vbuf, abuf, cbufv, cbufi;
  HIP_TRY(qbuf.alloc((size_t)(q_tiles_n * tile_bytes(ng)), s), "hipMallocAsync (queries)");
  float* binV = bins_val;
  int32_t* binA = bins_idx;
  if (!binV) {
    HIP_TRY(vbuf.alloc(sizeof(float) * (size_t)(M * L), s), "hipMallocAsync (bins)");
    binV = (float*)vbuf.p;
  }
  if (!binA) {
    HIP_TRY(abuf.alloc(sizeof(int32_t) * (size_t)(M * L), s), "hipMallocAsync (bins)");
    binA = (int32_t*)abuf.p;
  }
  HIP_TRY(launch_prepare(Q, q_dtype, M, db->D, db->metric, dt, false, (unsigned char*)qbuf.p, q_tiles_n, nullptr,
                         nullptr, s),
          "query preparation");
  FusedParams p{};
  p.db_tiles = db->tiles;
  p.q_tiles = (const unsigned char*)qbuf.p;
  p.N = db->N;
  p.L = L;
  p.M = M;
  p.bins_per_chunk = bpc;
  p.n_chunks = n_chunks;
  p.n_qb = (int32_t)n_qb;
  p.out_sign = db->metric == KNN_L2 ? -1.f : 1.f;
  p.binV = binV;
  p.binA = binA;
  p.ldo = L;
  HIP_TRY(launch_fused(dt, ng, ncb, p, s), "distance + bin-reduce kernel");
  const unsigned char* qt = (const unsigned char*)qbuf.p;
  if (bins_idx) HIP_TRY(launch_resolve(dt, binA, M, L, L, qt, db->tiles, ng, s), "resolve bin winners");
  const bool minimize = db->metric == KNN_L2;
  if (rerank_k <= 0) {
    HIP_TRY(launch_select(binV, binA, M, L, L, K, minimize, out_val, out_idx, K, s), "top-K select");
    HIP_TRY(launch_resolve(dt, out_idx, M, K, K, qt, db->tiles, ng, s), "resolve top-K rows");
    return KNN_OK;
  }
  HIP_TRY(cbufv.alloc(sizeof(float) * (size_t)(M * rerank_k), s), "hipMallocAsync (candidates)");
  HIP_TRY(cbufi.alloc(sizeof(int32_t) * (size_t)(M * rerank_k), s), "hipMallocAsync (candidates)");
  HIP_TRY(launch_select(binV, binA, M, L, L, rerank_k, minimize, (float*)cbufv.p, (int32_t*)cbufi.p, rerank_k, s),
          "top-K select (rerank candidates)");
  HIP_TRY(launch_resolve(dt, (int32_t*)cbufi.p, M, rerank_k, rerank_k, qt, db->tiles, ng, s),
          "resolve rerank candidates");
  HIP_TRY(launch_rerank((const int32_t*)cbufi.p, M, rerank_k, Q, q_dtype, db->X, db->in_dt, db->D, db->metric,
                        db->orig_half_norm, db->orig_rnorm, K, out_val, out_idx, s),
          "FP32 rerank");
  return KNN_OK;
}

extern "C" knn_status knn_db_search(const knn_db* db, const void* Q, int32_t q_dtype, int64_t M, int32_t K,
                                    int64_t L, int32_t rerank_k, float* out_val, int32_t* out_idx, float* bins_val,
                                    int32_t* bins_idx, void* stream) {
  g_last_error.clear();
  if (!db) return fail(KNN_ERR_INVALID, "db is NULL");
  if (L <= 0) L = knn_bins_for_recall(K, 0.95, db->N);
  knn_status st = check_sizes(M, db->N, db->D, K, L);
  if (st != KNN_OK) return st;
  if (!valid_in(q_dtype)) return fail(KNN_ERR_INVALID, "q_dtype must be KNN_F32 or KNN_BF16");
  if (M > 0 && (!Q || !out_val || !out_idx)) return fail(KNN_ERR_INVALID, "Q, out_val and out_idx must be non-NULL");
  if ((bins_val == nullptr) != (bins_idx == nullptr))
    return fail(KNN_ERR_INVALID, "bins_val and bins_idx must both be given or both be NULL");
  if (rerank_k != 0 && (rerank_k < K || rerank_k > L || rerank_k > 1024))
    return fail(KNN_ERR_INVALID, "rerank_k must be 0 or in [K, min(L, 1024)] (got %d)", rerank_k);
  if ((int64_t)M * L >= (int64_t(1) << 40)) return fail(KNN_ERR_UNSUPPORTED, "M * L too large");
  return search_core(db, Q, q_dtype, M, K, L, rerank_k, out_val, out_idx, bins_val, bins_idx, (hipStream_t)stream);
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
  DevBuf tiles;
  HIP_TRY(tiles.alloc((size_t)(db.n_tiles * tile_bytes(db.ng)), s), "hipMallocAsync (database)");
  db.tiles = (unsigned char*)tiles.p;
  HIP_TRY(launch_prepare(X, KNN_F32, N, D, metric, KNN_F32, true, db.tiles, db.n_tiles, nullptr, nullptr, s),
          "database preparation");
  return search_core(&db, Q, KNN_F32, M, K, L, 0, out_val, out_idx, nullptr, nullptr, s);
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

extern "C" knn_status knn_approx_top_k(const void* scores, int32_t dtype, int64_t rows, int64_t cols, int64_t ld,
                                       int32_t reduction_dim, int32_t K, double recall_target,
                                       int64_t input_size_override, int64_t L, int32_t minimize,
                                       int32_t aggregate_to_topk, float* out_val, int32_t* out_idx, void* stream) {
  g_last_error.clear();
  if (dtype != KNN_F32 && dtype != KNN_BF16) return fail(KNN_ERR_INVALID, "dtype must be KNN_F32 or KNN_BF16");
  if (rows < 0 || cols < 0) return fail(KNN_ERR_INVALID, "rows and cols must be >= 0");
  if (ld < cols || ld < 1) return fail(KNN_ERR_INVALID, "need ld >= max(cols, 1) (ld=%lld)", (long long)ld);
  if (reduction_dim == -1) reduction_dim = 1;
  if (reduction_dim != 0 && reduction_dim != 1) return fail(KNN_ERR_INVALID, "reduction_dim must be 0, 1 or -1");
  if (minimize != 0 && minimize != 1) return fail(KNN_ERR_INVALID, "minimize must be 0 or 1");
  if (aggregate_to_topk != 0 && aggregate_to_topk != 1) return fail(KNN_ERR_INVALID, "aggregate_to_topk must be 0 or 1");
  const int64_t n = reduction_dim == 1 ? cols : rows, B = reduction_dim == 1 ? rows : cols;
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
  if (B > 0 && (!scores || !out_val || !out_idx)) return fail(KNN_ERR_INVALID, "scores and outputs must be non-NULL");
  const size_t esz = dtype == KNN_F32 ? 4 : 2;
  if (reinterpret_cast<uintptr_t>(scores) % esz != 0) return fail(KNN_ERR_INVALID, "scores must be %zu-byte aligned", esz);
  if (B == 0) return KNN_OK;
  hipStream_t s = (hipStream_t)stream;
  const int dt = dtype == KNN_F32 ? DT_F32 : DT_BF16;
  if (!aggregate_to_topk) {
    HIP_TRY(launch_approx_bins(scores, dt, rows, cols, ld, reduction_dim, L, minimize != 0, out_val, out_idx, s),
            "approx bins");
    return KNN_OK;
  }
  DevBuf vbuf, abuf;
  HIP_TRY(vbuf.alloc(sizeof(float) * (size_t)(B * L), s), "hipMallocAsync (bins)");
  HIP_TRY(abuf.alloc(sizeof(int32_t) * (size_t)(B * L), s), "hipMallocAsync (bins)");
  float* V = static_cast<float*>(vbuf.p);
  int32_t* A = static_cast<int32_t*>(abuf.p);
  HIP_TRY(launch_approx_bins(scores, dt, rows, cols, ld, reduction_dim, L, minimize != 0, V, A, s), "approx bins");
  if (reduction_dim == 1)  // bins B x L, results B x K
    HIP_TRY(launch_select(V, A, B, L, L, K, minimize != 0, out_val, out_idx, K, s), "top-K");
  else  // bins L x B (bin-major), results K x B
    HIP_TRY(launch_select(V, A, B, L, 1, K, minimize != 0, out_val, out_idx, 1, s, B, B), "top-K");
  return KNN_OK;
}

// --------------------------------------------------------------------------- batched plan
namespace {

void free_plan_buffers(knn_plan* p) {
  for (auto& g : p->groups) {
    if (g.q_tiles) (void)hipFree(g.q_tiles);
    if (g.binV) (void)hipFree(g.binV);
    if (g.binA) (void)hipFree(g.binA);
    g.q_tiles = nullptr;
    g.binV = nullptr;
    g.binA = nullptr;
  }
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->d_groups) (void)hipFree(p->d_groups);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_sel) (void)hipFree(p->d_sel);
  p->d_segs = nullptr;
  p->d_groups = nullptr;
  p->d_items = nullptr;
  p->d_sel = nullptr;
}

// build (or rebuild after tuning) every device buffer and descriptor of the plan
knn_status build_plan_buffers(knn_plan* p, hipStream_t s) {
  free_plan_buffers(p);
  const int dt = p->compute;
  std::vector<QSeg> segs;
  std::vector<GroupDesc> gds;
  std::vector<SelRow> sel;
  int64_t first = 0;
  p->max_ng = 0;
  p->lds_bytes = 0;
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    GroupPlan& g = p->groups[gi];
    const knn_db* db = p->dbs[g.db];
    const int64_t QB = (int64_t)kWaves * 32 * g.ncb;
    g.n_qb = ceil_div(std::max<int64_t>(g.M, 1), QB);
    g.q_tiles_n = g.n_qb * QB / kTileRows;
    g.n_chunks = ceil_div(g.L, g.bins_per_chunk);
    p->max_ng = std::max(p->max_ng, db->ng);
    p->lds_bytes = std::max(p->lds_bytes, fused_lds_bytes(p->compute, db->ng, g.ncb));
    if (hipMalloc(&g.q_tiles, (size_t)(g.q_tiles_n * tile_bytes(db->ng))) != hipSuccess ||
        hipMalloc(&g.binV, sizeof(float) * (size_t)std::max<int64_t>(1, g.M * g.L)) != hipSuccess ||
        hipMalloc(&g.binA, sizeof(int32_t) * (size_t)std::max<int64_t>(1, g.M * g.L)) != hipSuccess)
      return fail(KNN_ERR_OOM, "hipMalloc for the batched plan");
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
      segs.push_back(q);
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
        sel.push_back(sr);
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
      segs.push_back(q);
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
    gds.push_back(gd);
  }
  p->total_q_rows = first;
  p->n_segs = (int)segs.size();
  p->n_sel_rows = (int64_t)sel.size();
  // work list: chunks dealt round-robin to the 8 XCDs; the items of one chunk
  // (all its query blocks) are consecutive in that XCD's list, so the persistent
  // workgroups of one XCD share a chunk's tiles through its L2
  std::vector<std::vector<WorkItem>> per_xcd(8);
  int64_t chunk_seq = 0;
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    const GroupPlan& g = p->groups[gi];
    if (g.M == 0) continue;
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
  const int blocks_per_xcd = 64;  // 2 resident workgroups on each of an XCD's 32 CUs
  p->n_blocks = 8 * blocks_per_xcd;
  size_t rounds = 0;
  for (auto& l : per_xcd) rounds = std::max<size_t>(rounds, (size_t)ceil_div((int64_t)l.size(), blocks_per_xcd));
  std::vector<WorkItem> items(rounds * p->n_blocks);
  for (size_t r = 0; r < rounds; ++r)
    for (int w = 0; w < p->n_blocks; ++w) {
      const int x = w % 8, i = w / 8;
      const size_t k = r * blocks_per_xcd + i;
      WorkItem it{};
      it.grp = -1;
      if (k < per_xcd[x].size()) it = per_xcd[x][k];
      items[r * p->n_blocks + w] = it;
    }
  p->n_items = (int64_t)items.size();
  if (hipMalloc(&p->d_segs, sizeof(QSeg) * std::max<size_t>(1, segs.size())) != hipSuccess ||
      hipMalloc(&p->d_groups, sizeof(GroupDesc) * std::max<size_t>(1, gds.size())) != hipSuccess ||
      hipMalloc(&p->d_items, sizeof(WorkItem) * std::max<size_t>(1, items.size())) != hipSuccess ||
      hipMalloc(&p->d_sel, sizeof(SelRow) * std::max<size_t>(1, sel.size())) != hipSuccess)
    return fail(KNN_ERR_OOM, "hipMalloc for the batched plan descriptors");
  HIP_TRY(hipMemcpyAsync(p->d_segs, segs.data(), sizeof(QSeg) * segs.size(), hipMemcpyHostToDevice, s), "upload");
  HIP_TRY(hipMemcpyAsync(p->d_groups, gds.data(), sizeof(GroupDesc) * gds.size(), hipMemcpyHostToDevice, s),
          "upload");
  HIP_TRY(hipMemcpyAsync(p->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, s),
          "upload");
  HIP_TRY(hipMemcpyAsync(p->d_sel, sel.data(), sizeof(SelRow) * sel.size(), hipMemcpyHostToDevice, s), "upload");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  return KNN_OK;
}

knn_status run_plan(knn_plan* p, hipStream_t s) {
  HIP_TRY(launch_prepare_segments(p->d_segs, p->n_segs, p->total_q_rows, p->q_dtype, p->compute, s),
          "batched query preparation");
  HIP_TRY(launch_fused_persistent(p->compute, p->d_groups, p->d_items, p->n_items, p->n_blocks, p->lds_bytes, s),
          "persistent distance + bin-reduce kernel");
  HIP_TRY(launch_select_rows(p->d_sel, p->n_sel_rows, p->max_K, s), "batched top-K select");
  HIP_TRY(launch_resolve_rows(p->compute, p->d_sel, p->n_sel_rows, s), "batched resolve");
  return KNN_OK;
}

// time one group alone with a given (ncb, L, bins_per_chunk), non-persistent launch
double time_group(knn_plan* p, size_t gi, hipStream_t s) {
  const GroupPlan& g = p->groups[gi];
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
  fp.out_sign = 1.f;
  fp.binV = g.binV;
  fp.binA = g.binA;
  fp.ldo = g.L;
  float* ov = nullptr;
  int32_t* oi = nullptr;
  if (hipMalloc(&ov, sizeof(float) * (size_t)(g.M * g.K_max)) != hipSuccess) return 1e30;
  if (hipMalloc(&oi, sizeof(int32_t) * (size_t)(g.M * g.K_max)) != hipSuccess) {
    (void)hipFree(ov);
    return 1e30;
  }
  hipEvent_t a, b;
  double best = 1e30;
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
      launch_prepare_segments(p->d_segs, p->n_segs, p->total_q_rows, p->q_dtype, p->compute, s) == hipSuccess &&
      launch_fused(db->compute, db->ng, g.ncb, fp, s) == hipSuccess) {  // warm-up
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(a, s);
      (void)launch_fused(db->compute, db->ng, g.ncb, fp, s);
      (void)launch_select(g.binV, g.binA, g.M, g.L, g.L, g.K_max, false, ov, oi, g.K_max, s);
      (void)hipEventRecord(b, s);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(ov);
  (void)hipFree(oi);
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
    << g.M << "|K" << g.K_max;
  return o.str();
}

// tiny JSON cache: {"key": [L, ncb, bins_per_chunk], ...}
std::map<std::string, std::vector<int64_t>> read_cache(const char* path) {
  std::map<std::string, std::vector<int64_t>> m;
  if (!path) return m;
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

void write_cache(const char* path, const std::map<std::string, std::vector<int64_t>>& m) {
  if (!path) return;
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

}  // namespace

extern "C" knn_status knn_plan_create(knn_db* const* dbs, int32_t ndb, const knn_batch* batches, int32_t nb,
                                      int32_t q_dtype, double recall_target, int32_t tune, const char* cache_path,
                                      void* stream, knn_plan** out) {
  g_last_error.clear();
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
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
  hipStream_t s = (hipStream_t)stream;
  auto* p = new (std::nothrow) knn_plan();
  if (!p) return fail(KNN_ERR_OOM, "host allocation");
  p->dbs.assign(dbs, dbs + ndb);
  p->batches.assign(batches, batches + nb);
  p->q_dtype = q_dtype;
  p->compute = compute;
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
    p->groups.push_back(g);
  }
  knn_status st = build_plan_buffers(p, s);
  if (st != KNN_OK) {
    knn_plan_destroy(p);
    return st;
  }
  if (tune) {
    auto cache = read_cache(cache_path);
    bool dirty = false;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
      GroupPlan& g = p->groups[gi];
      if (g.M == 0) continue;
      const std::string key = tune_key(p, g);
      auto it = cache.find(key);
      if (it != cache.end() && it->second.size() == 3) {
        g.L = it->second[0];
        g.ncb = (int32_t)it->second[1];
        g.bins_per_chunk = it->second[2];
        continue;
      }
      // candidates: L in {L_min, 2 L_min, 4 L_min, the L2-resident choice} (never
      // below the recall bound), ncb in {1, 2}, work-item sizes around the heuristic
      const int64_t N = dbs[g.db]->N;
      const int64_t Lmin = g.L_min;
      double best = 1e30;
      GroupPlan bestg = g;
      const int64_t Lfit = std::max(Lmin, bins_for_l2(N, dbs[g.db]->ng));
      for (int64_t Lc0 : {Lmin, 2 * Lmin, 4 * Lmin, Lfit}) {
        const int64_t Lc = std::min<int64_t>(N, Lc0);
        for (int ncb : {1, 2}) {
          if (!fused_supported(compute, dbs[g.db]->ng, ncb)) continue;
          const int64_t QB = (int64_t)kWaves * 32 * ncb;
          const int64_t nqb = ceil_div(g.M, QB);
          for (int64_t target : {int64_t(1024), int64_t(4096)}) {
            GroupPlan c = g;
            c.L = Lc;
            c.ncb = ncb;
            c.bins_per_chunk = pick_bins_per_chunk(N, Lc, nqb, dbs[g.db]->ng, target);
            p->groups[gi] = c;
            if (build_plan_buffers(p, s) != KNN_OK) continue;
            double ms = time_group(p, gi, s);
            if (ms < best) {
              best = ms;
              bestg = p->groups[gi];
            }
          }
        }
      }
      g = bestg;
      p->groups[gi] = bestg;
      cache[key] = {g.L, g.ncb, g.bins_per_chunk};
      dirty = true;
    }
    if (dirty) write_cache(cache_path, cache);
    st = build_plan_buffers(p, s);
    if (st != KNN_OK) {
      knn_plan_destroy(p);
      return st;
    }
  }
  *out = p;
  return KNN_OK;
}

extern "C" knn_status knn_search_batched(knn_plan* plan, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(KNN_ERR_INVALID, "plan is NULL");
  return run_plan(plan, (hipStream_t)stream);
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
  if (!plan) return KNN_OK;
  free_plan_buffers(plan);
  delete plan;
  return KNN_OK;
}
