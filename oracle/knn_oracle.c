/*
 * knn_oracle.c -- plain, slow FP64 reference for the approximate K-NN search
 * of "TPU-KNN: K Nearest Neighbor Search at Peak FLOP/s" (Chern et al., 2022).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (each function names the passage it follows):
 *   - scores: inner product (Sec. 2, eq. 2), relaxed squared-L2
 *     1/2|x|^2 - <q,x> (Appendix "Euclidean distance search", eq. l2final),
 *     cosine similarity <q,x>/(|q||x|) (Sec. 2, cosine distance definition);
 *   - the bin-wise partial reduction of Algorithm 1 (PartialReduce): in each
 *     of L bins keep the best score and its index, scanning rows in increasing
 *     order and replacing only on a strictly better score;
 *   - the exact top-K over the bin winners (the ExactRescoring step, Sec. 5);
 *   - the exact K-NN ground truth (eq. 1 / eq. 2) by a full sort of all N scores.
 *
 * Readings of the paper taken here (the paper leaves these open):
 *   - bins are contiguous balanced row ranges: bin b = [floor(bN/L), floor((b+1)N/L));
 *     when N = L * 2^W this is exactly ShiftRight(j, W) of Algorithm 1;
 *   - rows and bins are numbered from 0;
 *   - ties inside a bin go to the lowest row index (strict comparison in
 *     increasing row order); ties in a top-K go to the lowest index;
 *   - "better" is larger for MIPS and cosine, smaller for relaxed L2;
 *   - a zero-norm vector has cosine similarity 0 with everything.
 *
 * Inputs are FP32 arrays; every product of two FP32 values is exact in FP64
 * (48 significant bits), so the FP64 sums are the reference scores.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_MIPS = 0, OR_L2 = 1, OR_COSINE = 2 };

typedef struct {
  double v;
  int64_t j;
} or_pair;

/* First row of bin b under the contiguous balanced partition. */
int64_t or_bin_start(int64_t b, int64_t N, int64_t L) {
  return (int64_t)(((__int128)b * (__int128)N) / (__int128)L);
}

/* Bin that holds row j: the largest b with or_bin_start(b) <= j. */
int64_t or_bin_of(int64_t j, int64_t N, int64_t L) {
  int64_t lo = 0, hi = L - 1;
  while (lo < hi) { /* plain bisection on the definition of the bin ranges */
    int64_t mid = (lo + hi + 1) / 2;
    if (or_bin_start(mid, N, L) <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* is score a strictly better than score b? */
static int better(double a, double b, int minimize) { return minimize ? (a < b) : (a > b); }

/* Score of one (query, row) pair in FP64, and the magnitude sum that bounds its
 * rounding error in any FP32 summation order (sum |q_k x_k|, plus 1/2 sum x_k^2
 * for L2; for cosine the normalised form plus one unit for the normalisation). */
static double or_score1(const float* q, const float* x, int32_t D, int32_t metric, double* mag) {
  double dot = 0.0, absdot = 0.0, qq = 0.0, xx = 0.0;
  for (int32_t k = 0; k < D; ++k) {
    double a = (double)q[k], b = (double)x[k];
    dot += a * b;
    absdot += fabs(a * b);
    qq += a * a;
    xx += b * b;
  }
  if (metric == OR_MIPS) {
    if (mag) *mag = absdot;
    return dot;
  }
  if (metric == OR_L2) {
    if (mag) *mag = absdot + 0.5 * xx;
    return 0.5 * xx - dot;
  }
  /* cosine similarity */
  double nq = sqrt(qq), nx = sqrt(xx);
  if (nq == 0.0 || nx == 0.0) {
    if (mag) *mag = 1.0;
    return 0.0;
  }
  if (mag) *mag = absdot / (nq * nx) + 1.0;
  return dot / (nq * nx);
}

void or_pair_scores(const float* Q, const float* X, int32_t D, int32_t metric, const int64_t* qi,
                    const int64_t* xj, int64_t n, double* out_s, double* out_mag) {
  for (int64_t t = 0; t < n; ++t) {
    double mag = 0.0;
    double s = or_score1(Q + qi[t] * (int64_t)D, X + xj[t] * (int64_t)D, D, metric, &mag);
    out_s[t] = s;
    if (out_mag) out_mag[t] = mag;
  }
}

/* Full score matrix S[M x N] (only for small problems). */
void or_scores(const float* Q, const float* X, int64_t M, int64_t N, int32_t D, int32_t metric, double* S,
               double* MAG) {
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      double mag = 0.0;
      S[i * N + j] = or_score1(Q + i * (int64_t)D, X + j * (int64_t)D, D, metric, &mag);
      if (MAG) MAG[i * N + j] = mag;
    }
}

static int cmp_desc(const void* pa, const void* pb) {
  const or_pair* a = (const or_pair*)pa;
  const or_pair* b = (const or_pair*)pb;
  if (a->v > b->v) return -1;
  if (a->v < b->v) return 1;
  return (a->j < b->j) ? -1 : (a->j > b->j);
}
static int cmp_asc(const void* pa, const void* pb) {
  const or_pair* a = (const or_pair*)pa;
  const or_pair* b = (const or_pair*)pb;
  if (a->v < b->v) return -1;
  if (a->v > b->v) return 1;
  return (a->j < b->j) ? -1 : (a->j > b->j);
}

/* Sort the pairs best-first (ties: lowest index first). */
static void sort_pairs(or_pair* p, int64_t n, int minimize) {
  qsort(p, (size_t)n, sizeof(or_pair), minimize ? cmp_asc : cmp_desc);
}

/* Algorithm 1 on one row of scores s[0..N): for every bin, the best score, its
 * row and magnitude; and, for the tests' tolerance, the best score among the
 * bin's other rows (V2) and the largest magnitude among those other rows (V2M).
 * A winner that is ahead of V2 by more than the rounding bound of its own
 * magnitude plus V2M is then ahead of every other row of the bin by more than
 * the bound of the two scores, whatever their individual magnitudes. */
static void partial_reduce_row(const double* s, const double* mag, int64_t N, int64_t L, int minimize,
                               double* V, int64_t* A, double* VM, double* V2, double* V2M) {
  const double worst = minimize ? INFINITY : -INFINITY;
  for (int64_t b = 0; b < L; ++b) {
    int64_t j0 = or_bin_start(b, N, L), j1 = or_bin_start(b + 1, N, L);
    double v = worst, v2 = worst, vm = 0.0, v2m = 0.0;
    int64_t a = -1;
    for (int64_t j = j0; j < j1; ++j) {
      double y = s[j];
      double m = mag ? mag[j] : 0.0;
      if (better(y, v, minimize)) { /* the compare and the two conditional moves */
        if (a >= 0) {                 /* the old winner joins the other rows */
          v2 = v;                     /* it was at least as good as all of them */
          if (vm > v2m) v2m = vm;
        }
        v = y;
        vm = m;
        a = j;
      } else {                        /* row j is not the winner at this point, nor later */
        if (better(y, v2, minimize)) v2 = y;
        if (m > v2m) v2m = m;
      }
    }
    V[b] = v;
    A[b] = a;
    if (VM) VM[b] = vm;
    if (V2) V2[b] = v2;
    if (V2M) V2M[b] = v2m;
  }
}

/* PartialReduce on a given score matrix S[M x N] (row-major). */
void or_partial_reduce(const double* S, int64_t M, int64_t N, int64_t L, int32_t minimize, double* V,
                       int64_t* A) {
  for (int64_t i = 0; i < M; ++i)
    partial_reduce_row(S + i * N, NULL, N, L, minimize, V + i * L, A + i * L, NULL, NULL, NULL);
}

/* Exact top-K of n candidate pairs (values v, indices a): full sort, keep K. */
void or_topk_pairs(const double* v, const int64_t* a, int64_t M, int64_t n, int32_t K, int32_t minimize,
                   double* outV, int64_t* outA) {
  or_pair* p = (or_pair*)malloc(sizeof(or_pair) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t t = 0; t < n; ++t) {
      p[t].v = v[i * n + t];
      p[t].j = a[i * n + t];
    }
    sort_pairs(p, n, minimize);
    for (int32_t k = 0; k < K; ++k) {
      outV[i * K + k] = (k < n) ? p[k].v : NAN;
      outA[i * K + k] = (k < n) ? p[k].j : -1;
    }
  }
  free(p);
}

/*
 * The whole approximate search per query, without materialising S for more
 * than one query at a time:
 *   scores -> Algorithm 1 bins -> exact top-K of the L bin winners,
 * and optionally the exact K-NN by a full sort of the N scores.
 * Any output pointer may be NULL.  Bin outputs are M x L, top-K outputs M x K.
 * Returns 0, or -1 on invalid sizes.
 */
int or_search(const float* Q, const float* X, int64_t M, int64_t N, int32_t D, int32_t metric, int64_t L,
              int32_t K, double* binV, int64_t* binA, double* binMag, double* bin2V, double* bin2Mag,
              double* topV, int64_t* topA, double* exV, int64_t* exA, int32_t nthreads) {
  if (M < 0 || N < 1 || D < 1 || L < 1 || L > N || K < 1 || K > L) return -1;
  const int minimize = (metric == OR_L2);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    double* s = (double*)malloc(sizeof(double) * (size_t)N);
    double* mag = (double*)malloc(sizeof(double) * (size_t)N);
    double* V = (double*)malloc(sizeof(double) * (size_t)L);
    int64_t* A = (int64_t*)malloc(sizeof(int64_t) * (size_t)L);
    double* VM = (double*)malloc(sizeof(double) * (size_t)L);
    double* V2 = (double*)malloc(sizeof(double) * (size_t)L);
    double* V2M = (double*)malloc(sizeof(double) * (size_t)L);
    or_pair* p = (or_pair*)malloc(sizeof(or_pair) * (size_t)(exV || exA ? N : L));
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i) {
      const float* q = Q + i * (int64_t)D;
      for (int64_t j = 0; j < N; ++j) s[j] = or_score1(q, X + j * (int64_t)D, D, metric, &mag[j]);
      partial_reduce_row(s, mag, N, L, minimize, V, A, VM, V2, V2M);
      if (binV) memcpy(binV + i * L, V, sizeof(double) * (size_t)L);
      if (binA) memcpy(binA + i * L, A, sizeof(int64_t) * (size_t)L);
      if (binMag) memcpy(binMag + i * L, VM, sizeof(double) * (size_t)L);
      if (bin2V) memcpy(bin2V + i * L, V2, sizeof(double) * (size_t)L);
      if (bin2Mag) memcpy(bin2Mag + i * L, V2M, sizeof(double) * (size_t)L);
      if (topV || topA) {
        for (int64_t b = 0; b < L; ++b) {
          p[b].v = V[b];
          p[b].j = A[b];
        }
        sort_pairs(p, L, minimize);
        for (int32_t k = 0; k < K; ++k) {
          if (topV) topV[i * K + k] = p[k].v;
          if (topA) topA[i * K + k] = p[k].j;
        }
      }
      if (exV || exA) {
        for (int64_t j = 0; j < N; ++j) {
          p[j].v = s[j];
          p[j].j = j;
        }
        sort_pairs(p, N, minimize);
        for (int32_t k = 0; k < K; ++k) {
          if (exV) exV[i * K + k] = p[k].v;
          if (exA) exA[i * K + k] = p[k].j;
        }
      }
    }
    free(s);
    free(mag);
    free(V);
    free(A);
    free(VM);
    free(V2);
    free(V2M);
    free(p);
  }
  return 0;
}

/*
 * Dense FP64 reference gradient of sum_{i,k} g[i,k] * score(q_i, x_{a[i,k]})
 * with the selection a held fixed: scatter g into an M x N matrix G and form
 * dQ = dS/dq contracted with G, dX likewise (for MIPS dQ = G X, dX = G^T Q).
 * Score derivatives: MIPS d<q,x>/dq = x, /dx = q; relaxed L2
 * (1/2|x|^2 - <q,x>): /dq = -x, /dx = x - q; cosine c = <q,x>/(|q||x|):
 * /dq = x/(|q||x|) - c q/|q|^2, /dx = q/(|q||x|) - c x/|x|^2.
 * dQ is M x D and dX is N x D, both overwritten.
 */
void or_backward(const double* g, const int64_t* a, const float* Q, const float* X, int64_t M, int64_t N,
                 int32_t D, int32_t K, int32_t metric, double* dQ, double* dX) {
  memset(dQ, 0, sizeof(double) * (size_t)(M * D));
  memset(dX, 0, sizeof(double) * (size_t)(N * D));
  for (int64_t i = 0; i < M; ++i) {
    const float* q = Q + i * (int64_t)D;
    double qq = 0.0;
    for (int32_t d = 0; d < D; ++d) qq += (double)q[d] * (double)q[d];
    for (int32_t k = 0; k < K; ++k) {
      int64_t j = a[i * K + k];
      if (j < 0 || j >= N) continue;
      double gk = g[i * K + k];
      const float* x = X + j * (int64_t)D;
      if (metric == OR_MIPS) {
        for (int32_t d = 0; d < D; ++d) {
          dQ[i * D + d] += gk * (double)x[d];
          dX[j * D + d] += gk * (double)q[d];
        }
      } else if (metric == OR_L2) {
        for (int32_t d = 0; d < D; ++d) {
          dQ[i * D + d] -= gk * (double)x[d];
          dX[j * D + d] += gk * ((double)x[d] - (double)q[d]);
        }
      } else {
        double xx = 0.0, dot = 0.0;
        for (int32_t d = 0; d < D; ++d) {
          xx += (double)x[d] * (double)x[d];
          dot += (double)q[d] * (double)x[d];
        }
        double nq = sqrt(qq), nx = sqrt(xx);
        if (nq == 0.0 || nx == 0.0) continue;
        double c = dot / (nq * nx);
        for (int32_t d = 0; d < D; ++d) {
          dQ[i * D + d] += gk * ((double)x[d] / (nq * nx) - c * (double)q[d] / qq);
          dX[j * D + d] += gk * ((double)q[d] / (nq * nx) - c * (double)x[d] / xx);
        }
      }
    }
  }
}
