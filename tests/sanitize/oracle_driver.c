/*
 * Drives every exported function of the C oracle (oracle/knn_oracle.c) over small
 * inputs and edge shapes, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Any out-of-bounds access,
 * use of freed memory, signed overflow or misaligned access aborts the run.
 * Exit status 0: every call returned and the results passed the checks below.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t or_bin_start(int64_t b, int64_t N, int64_t L);
int64_t or_bin_of(int64_t j, int64_t N, int64_t L);
void or_pair_scores(const float* Q, const float* X, int32_t D, int32_t metric, const int64_t* qi,
                    const int64_t* xj, int64_t n, double* out_s, double* out_mag);
void or_scores(const float* Q, const float* X, int64_t M, int64_t N, int32_t D, int32_t metric, double* S,
               double* MAG);
void or_partial_reduce(const double* S, int64_t M, int64_t N, int64_t L, int32_t minimize, double* V,
                       int64_t* A);
void or_topk_pairs(const double* v, const int64_t* a, int64_t M, int64_t n, int32_t K, int32_t minimize,
                   double* outV, int64_t* outA);
int or_search(const float* Q, const float* X, int64_t M, int64_t N, int32_t D, int32_t metric, int64_t L,
              int32_t K, double* binV, int64_t* binA, double* binMag, double* bin2V, double* bin2Mag,
              double* topV, int64_t* topA, double* exV, int64_t* exA, int32_t nthreads);
void or_backward(const double* g, const int64_t* a, const float* Q, const float* X, int64_t M, int64_t N,
                 int32_t D, int32_t K, int32_t metric, double* dQ, double* dX);

static uint64_t rng = 88172645463325252ull;
static float next_val(int ints) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  if (ints) return (float)((int)(rng % 9u) - 4);  // many exact ties
  return (float)((double)(rng >> 11) / 9007199254740992.0 * 2.0 - 1.0);
}

static int failures = 0;
#define CHECK(c, ...)                   \
  do {                                  \
    if (!(c)) {                         \
      fprintf(stderr, __VA_ARGS__);     \
      fprintf(stderr, "\n");            \
      ++failures;                       \
    }                                   \
  } while (0)

static void run_case(int64_t M, int64_t N, int32_t D, int64_t L, int32_t K, int32_t metric, int ints) {
  float* Q = malloc(sizeof(float) * (size_t)(M * D));
  float* X = malloc(sizeof(float) * (size_t)(N * D));
  for (int64_t i = 0; i < M * D; ++i) Q[i] = next_val(ints);
  for (int64_t i = 0; i < N * D; ++i) X[i] = next_val(ints);
  if (N > 1) for (int32_t d = 0; d < D; ++d) X[d] = 0.f;  // a zero row (cosine: similarity 0)
  double* binV = malloc(sizeof(double) * (size_t)(M * L));
  int64_t* binA = malloc(sizeof(int64_t) * (size_t)(M * L));
  double* binMag = malloc(sizeof(double) * (size_t)(M * L));
  double* bin2V = malloc(sizeof(double) * (size_t)(M * L));
  double* bin2Mag = malloc(sizeof(double) * (size_t)(M * L));
  double* topV = malloc(sizeof(double) * (size_t)(M * K));
  int64_t* topA = malloc(sizeof(int64_t) * (size_t)(M * K));
  double* exV = malloc(sizeof(double) * (size_t)(M * K));
  int64_t* exA = malloc(sizeof(int64_t) * (size_t)(M * K));
  int rc = or_search(Q, X, M, N, D, metric, L, K, binV, binA, binMag, bin2V, bin2Mag, topV, topA, exV, exA, 1);
  CHECK(rc == 0, "or_search rc %d (M=%lld N=%lld L=%lld K=%d)", rc, (long long)M, (long long)N, (long long)L, K);
  const int minimize = metric == 1;
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t b = 0; b < L; ++b) {
      const int64_t j = binA[i * L + b];
      CHECK(j >= or_bin_start(b, N, L) && j < or_bin_start(b + 1, N, L), "bin winner outside its bin");
      CHECK(or_bin_of(j, N, L) == b, "or_bin_of disagrees with or_bin_start");
    }
    for (int32_t k = 1; k < K; ++k) {
      const double a = topV[i * K + k - 1], c = topV[i * K + k];
      CHECK(minimize ? a <= c : a >= c, "top-K not ordered");
    }
  }
  /* the full score matrix, bins and top-K from it agree with or_search */
  double* S = malloc(sizeof(double) * (size_t)(M * N));
  double* MAG = malloc(sizeof(double) * (size_t)(M * N));
  or_scores(Q, X, M, N, D, metric, S, MAG);
  double* V2 = malloc(sizeof(double) * (size_t)(M * L));
  int64_t* A2 = malloc(sizeof(int64_t) * (size_t)(M * L));
  or_partial_reduce(S, M, N, L, minimize, V2, A2);
  for (int64_t t = 0; t < M * L; ++t) CHECK(A2[t] == binA[t] && V2[t] == binV[t], "or_partial_reduce differs");
  double* tv = malloc(sizeof(double) * (size_t)(M * K));
  int64_t* ta = malloc(sizeof(int64_t) * (size_t)(M * K));
  or_topk_pairs(V2, A2, M, L, K, minimize, tv, ta);
  for (int64_t t = 0; t < M * K; ++t) CHECK(ta[t] == topA[t], "or_topk_pairs differs");
  /* pair scores on the winners */
  int64_t* qi = malloc(sizeof(int64_t) * (size_t)(M * K));
  for (int64_t t = 0; t < M * K; ++t) qi[t] = t / K;
  double* ps = malloc(sizeof(double) * (size_t)(M * K));
  double* pm = malloc(sizeof(double) * (size_t)(M * K));
  or_pair_scores(Q, X, D, metric, qi, topA, M * K, ps, pm);
  for (int64_t t = 0; t < M * K; ++t) CHECK(ps[t] == topV[t], "or_pair_scores differs");
  /* backward through the top-K (one index out of range is skipped) */
  double* g = malloc(sizeof(double) * (size_t)(M * K));
  for (int64_t t = 0; t < M * K; ++t) g[t] = next_val(0);
  int64_t* a = malloc(sizeof(int64_t) * (size_t)(M * K));
  for (int64_t t = 0; t < M * K; ++t) a[t] = topA[t];
  if (M * K > 0) a[0] = -1;
  double* dQ = malloc(sizeof(double) * (size_t)(M * D));
  double* dX = malloc(sizeof(double) * (size_t)(N * D));
  or_backward(g, a, Q, X, M, N, D, K, metric, dQ, dX);
  for (int64_t t = 0; t < M * D; ++t) CHECK(!isnan(dQ[t]), "dQ NaN");
  free(Q); free(X); free(binV); free(binA); free(binMag); free(bin2V); free(bin2Mag); free(topV); free(topA);
  free(exV); free(exA); free(S); free(MAG); free(V2); free(A2); free(tv); free(ta); free(qi); free(ps); free(pm);
  free(g); free(a); free(dQ); free(dX);
}

int main(void) {
  for (int32_t metric = 0; metric < 3; ++metric) {
    run_case(5, 97, 7, 13, 4, metric, 0);    /* bins of 7-8 rows */
    run_case(3, 64, 16, 64, 10, metric, 1);  /* L = N: one row per bin, integer ties */
    run_case(4, 50, 3, 5, 5, metric, 1);     /* K = L */
    run_case(1, 1, 1, 1, 1, metric, 0);      /* one row */
    run_case(2, 33, 1, 2, 1, metric, 1);     /* D = 1 */
    run_case(0, 10, 4, 3, 2, metric, 0);     /* no queries */
  }
  CHECK(or_search(NULL, NULL, 1, 10, 4, 0, 11, 1, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 1) == -1,
        "L > N accepted");
  CHECK(or_search(NULL, NULL, 1, 10, 4, 0, 5, 6, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 1) == -1,
        "K > L accepted");
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle driver: all calls clean\n");
  return 0;
}
