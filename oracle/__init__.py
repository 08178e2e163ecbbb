"""Plain CPU oracle for the approximate K-NN search of TPU-KNN (Chern et al., 2022).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product path never does.  It shares
no code with the HIP library.

Parts:
  * ``knn_oracle.c`` (FP64, OpenMP over queries): scores, Algorithm 1
    (PartialReduce) on contiguous balanced bins, exact top-K of the bin
    winners, exact K-NN by full sort, dense reference gradients.
  * ``approx_top_k`` / ``approx_bins``: the approx_max_k op of App. A.1 on a given
    score matrix (Algorithm 1 along either dimension, optional top-K, the bin count
    from the recall target and the input-size override).
  * this module: the ctypes wrapper for it, the recall model of Sec. 5.1
    (eq. recall, eq. l:approx and the appendix on the number of bins), the
    exact recall expectation for fixed balanced bins, recall metrics
    (eq. recall-def) and the reference quantisers (BF16 round-to-nearest-even,
    FP8 E4M3 with a power-of-two scale per row) written from the definitions
    of the formats.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.c")
_LIB = os.path.join(_HERE, "libknn_oracle.so")
_lib = None

MIPS, L2, COSINE = 0, 1, 2
METRICS = {"mips": MIPS, "l2": L2, "cosine": COSINE}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC])
    return _LIB


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.or_bin_start.restype = i64
        lib.or_bin_start.argtypes = [i64, i64, i64]
        lib.or_bin_of.restype = i64
        lib.or_bin_of.argtypes = [i64, i64, i64]
        lib.or_pair_scores.restype = None
        lib.or_pair_scores.argtypes = [P, P, i32, i32, P, P, i64, P, P]
        lib.or_scores.restype = None
        lib.or_scores.argtypes = [P, P, i64, i64, i32, i32, P, P]
        lib.or_partial_reduce.restype = None
        lib.or_partial_reduce.argtypes = [P, i64, i64, i64, i32, P, P]
        lib.or_topk_pairs.restype = None
        lib.or_topk_pairs.argtypes = [P, P, i64, i64, i32, i32, P, P]
        lib.or_search.restype = ctypes.c_int
        lib.or_search.argtypes = [P, P, i64, i64, i32, i32, i64, i32] + [P] * 9 + [i32]
        lib.or_backward.restype = None
        lib.or_backward.argtypes = [P, P, P, P, i64, i64, i32, i32, i32, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _metric(m):
    return METRICS[m] if isinstance(m, str) else int(m)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ----------------------------------------------------------------------------------------
# bins (Algorithm 1 with contiguous balanced bins)
# ----------------------------------------------------------------------------------------
def bin_start(b: int, N: int, L: int) -> int:
    """First row of bin b: floor(b*N/L)."""
    return int(_get().or_bin_start(int(b), int(N), int(L)))


def bin_of(j: int, N: int, L: int) -> int:
    return int(_get().or_bin_of(int(j), int(N), int(L)))


def minimize_for(metric) -> bool:
    """Relaxed L2 is minimised; MIPS and cosine similarity are maximised."""
    return _metric(metric) == L2


def scores(Q, X, metric):
    """Full FP64 score matrix S[M x N] and the rounding magnitudes (small inputs only)."""
    Q, X = _f32(Q), _f32(X)
    M, D = Q.shape
    N = X.shape[0]
    S = np.empty((M, N), np.float64)
    MAG = np.empty((M, N), np.float64)
    _get().or_scores(_p(Q), _p(X), M, N, D, _metric(metric), _p(S), _p(MAG))
    return S, MAG


def pair_scores(Q, X, metric, qi, xj):
    """FP64 scores (and magnitudes) of the listed (query, row) pairs."""
    Q, X = _f32(Q), _f32(X)
    qi = np.ascontiguousarray(qi, np.int64).ravel()
    xj = np.ascontiguousarray(xj, np.int64).ravel()
    s = np.empty(qi.size, np.float64)
    mag = np.empty(qi.size, np.float64)
    _get().or_pair_scores(_p(Q), _p(X), Q.shape[1], _metric(metric), _p(qi), _p(xj), qi.size, _p(s), _p(mag))
    return s, mag


def partial_reduce(S, L: int, minimize: bool):
    """Algorithm 1 on a given score matrix: bin winners V[M x L] and their rows A[M x L]."""
    S = np.ascontiguousarray(S, np.float64)
    M, N = S.shape
    V = np.empty((M, L), np.float64)
    A = np.empty((M, L), np.int64)
    _get().or_partial_reduce(_p(S), M, N, L, int(minimize), _p(V), _p(A))
    return V, A


def topk_pairs(v, a, K: int, minimize: bool):
    """Exact top-K of candidate (value, index) pairs per row: full sort, best first, ties to the lower index."""
    v = np.ascontiguousarray(v, np.float64)
    a = np.ascontiguousarray(a, np.int64)
    M, n = v.shape
    oV = np.empty((M, K), np.float64)
    oA = np.empty((M, K), np.int64)
    _get().or_topk_pairs(_p(v), _p(a), M, n, K, int(minimize), _p(oV), _p(oA))
    return oV, oA


def search(Q, X, metric, L: int, K: int, *, bins: bool = False, exact: bool = False, nthreads: int = 0):
    """Approximate search of the paper (scores -> Algorithm 1 -> top-K of the bins), in FP64.

    Returns a dict with ``top_v``/``top_i`` (M x K), and with ``bins=True`` the bin winners
    ``bin_v``/``bin_i``/``bin_mag`` (M x L), the best score among each bin's other rows
    ``bin2_v`` and the largest magnitude among those other rows ``bin2_mag``; with
    ``exact=True`` the exact K-NN ``ex_v``/``ex_i`` (M x K) by a full sort of all N scores.
    """
    Q, X = _f32(Q), _f32(X)
    M, D = Q.shape
    N = X.shape[0]
    assert X.shape[1] == D
    out = {"top_v": np.empty((M, K)), "top_i": np.empty((M, K), np.int64)}
    if bins:
        for k in ("bin_v", "bin_mag", "bin2_v", "bin2_mag"):
            out[k] = np.empty((M, L))
        out["bin_i"] = np.empty((M, L), np.int64)
    if exact:
        out["ex_v"] = np.empty((M, K))
        out["ex_i"] = np.empty((M, K), np.int64)
    g = out.get
    rc = _get().or_search(_p(Q), _p(X), M, N, D, _metric(metric), L, K, _p(g("bin_v")), _p(g("bin_i")),
                          _p(g("bin_mag")), _p(g("bin2_v")), _p(g("bin2_mag")), _p(out["top_v"]),
                          _p(out["top_i"]), _p(g("ex_v")), _p(g("ex_i")), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid sizes (need 1 <= K <= L <= N, D >= 1)")
    return out


def approx_bins(n: int, K: int, r: float = 0.95, input_size_override: int = -1) -> int:
    """Bins of the approx_max_k op for a slice of n scores (App. A.1's options): the recall
    target fixes L for the evaluated size (eq. l:approx, exact inverse); a positive
    ``input_size_override`` evaluates that size instead and keeps its bin density for the
    n scores at hand, L = ceil(L_eval * n / override) (the reading used for shards of a
    longer reduction); clamped to [K, n]."""
    n_eval = input_size_override if input_size_override > 0 else n
    L = bins_for_recall(K, r, n_eval)
    if input_size_override > 0:
        L = -((-L * n) // n_eval)
    return min(max(L, K), n)


def approx_top_k(S, K: int, L: int, dim: int = -1, minimize: bool = False, aggregate: bool = True):
    """The approx_max_k / approx_min_k op on a given score matrix (App. A.1): Algorithm 1
    over each slice along ``dim`` (rows for dim = 1 or -1, columns for dim = 0), then,
    with ``aggregate``, the exact top-K of the bin winners (ExactRescoring).  The result
    keeps the input's layout with the reduced dimension replaced by K (or L); indices are
    positions along the reduced dimension.  Scores are widened to FP64 exactly."""
    S = np.asarray(S, np.float64)
    T = S if dim in (-1, 1) else S.T
    B, n = T.shape
    V = np.empty((B, L))
    A = np.empty((B, L), np.int64)
    rows = np.arange(B)
    for b in range(L):
        # bin b: positions [floor(b n / L), floor((b + 1) n / L)); numpy's argmax / argmin
        # return the first best position, i.e. the strict comparison scanning upwards.
        # The bin's first score starts the scan, so a bin of -inf scores (masked-out
        # entries) still reports its first position.
        j0, j1 = (b * n) // L, ((b + 1) * n) // L
        blk = T[:, j0:j1]
        a = np.argmin(blk, axis=1) if minimize else np.argmax(blk, axis=1)
        V[:, b] = blk[rows, a]
        A[:, b] = j0 + a
    if aggregate:
        V, A = topk_pairs(V, A, K, minimize)
    if dim == 0:
        V, A = V.T, A.T
    return np.ascontiguousarray(V), np.ascontiguousarray(A)


def backward(g, a, Q, X, metric):
    """Dense FP64 gradient of sum g[i,k]*score(q_i, x_{a[i,k]}) with the selection held fixed."""
    Q, X = _f32(Q), _f32(X)
    g = np.ascontiguousarray(g, np.float64)
    a = np.ascontiguousarray(a, np.int64)
    M, D = Q.shape
    N = X.shape[0]
    K = g.shape[1]
    dQ = np.empty((M, D))
    dX = np.empty((N, D))
    _get().or_backward(_p(g), _p(a), _p(Q), _p(X), M, N, D, K, _metric(metric), _p(dQ), _p(dX))
    return dQ, dX


# ----------------------------------------------------------------------------------------
# recall model (Sec. 5.1 and the appendix on the number of bins)
# ----------------------------------------------------------------------------------------
def recall_bound_paper(K: int, L: int) -> float:
    """eq. recall: E[Z]/K = ((L-1)/L)^(K-1), Z = balls alone in their bin."""
    return ((L - 1) / L) ** (K - 1)


def bins_for_recall(K: int, r: float, N: int | None = None) -> int:
    """Smallest L with ((L-1)/L)^(K-1) >= r (eq. l:approx, exact inverse), clamped to [K, N].

    K = 1 needs a single bin: the global best is always some bin's winner.
    """
    if K <= 1:
        L = 1
    else:
        L = math.ceil(1.0 / (1.0 - r ** (1.0 / (K - 1))))
        # guard the ceiling against rounding of the closed form
        while L > 1 and recall_bound_paper(K, L - 1) >= r:
            L -= 1
        while recall_bound_paper(K, L) < r:
            L += 1
    L = max(L, K)
    if N is not None:
        L = min(L, N)
    return L


def bins_for_recall_approx(K: int, r: float) -> float:
    """The first-order form of eq. l:approx: L ~ (K-1)/(1-r)."""
    return (K - 1) / (1.0 - r)


def recall_exact_balanced(N: int, L: int, K: int, exact_fraction: bool = False):
    """E[recall] when the K true neighbours sit at a uniformly random K-subset of the N rows.

    Every bin that holds at least one of them contributes exactly one retrieved neighbour
    (its winner), so recall = (#occupied bins)/K and
    E = (1/K) sum_b [1 - C(N-B_b, K)/C(N, K)], B_b the size of bin b.
    """
    sizes = [bin_start(b + 1, N, L) - bin_start(b, N, L) for b in range(L)] if L <= 200000 else None
    if exact_fraction:
        tot = math.comb(N, K)
        acc = Fraction(0)
        for B in sizes:
            acc += 1 - Fraction(math.comb(N - B, K), tot)
        return acc / K
    from collections import Counter
    acc = 0.0
    for B, cnt in Counter(sizes).items():
        p_empty = 1.0
        for t in range(K):
            p_empty *= max(N - B - t, 0) / (N - t)
        acc += cnt * (1.0 - p_empty)
    return acc / K


def recall_independent(L: int, K: int) -> float:
    """E[#occupied bins]/K for K balls placed independently and uniformly: L(1-(1-1/L)^K)/K."""
    return L * (1.0 - (1.0 - 1.0 / L) ** K) / K


def recall(retrieved, truth) -> np.ndarray:
    """eq. recall-def per query: |S_q intersect S*_q| / |S*_q|."""
    retrieved = np.asarray(retrieved)
    truth = np.asarray(truth)
    out = np.empty(truth.shape[0])
    for i in range(truth.shape[0]):
        out[i] = len(set(retrieved[i].tolist()) & set(truth[i].tolist())) / truth.shape[1]
    return out


def recall_tie_aware(retrieved_scores, exact_scores, minimize: bool) -> np.ndarray:
    """eq. recall-def when the exact K-NN is not unique (ties at the K-th score).

    Any set of K rows that scores at least as well as every row left out is an exact
    K-NN; the recall of a retrieved set S (K distinct rows, given by their exact
    scores) is its best overlap with such a set, divided by K.  With s_K the K-th best
    exact score and B the rows strictly better than s_K (all of them are among the
    exact top K), every exact K-NN is B plus K - |B| of the rows tied at s_K, so the
    best overlap is |S among B| + min(|S tied at s_K|, K - |B|).
    ``exact_scores``: the exact top-K scores of each query, best first (M x K)."""
    rs = np.asarray(retrieved_scores, np.float64)
    ex = np.asarray(exact_scores, np.float64)
    K = ex.shape[1]
    sK = ex[:, K - 1:K]
    strictly = (lambda a: a < sK) if minimize else (lambda a: a > sK)
    n_b = strictly(ex).sum(axis=1)
    hit_b = strictly(rs).sum(axis=1)
    hit_tie = (rs == sK).sum(axis=1)
    return (hit_b + np.minimum(hit_tie, K - n_b)) / K


# ----------------------------------------------------------------------------------------
# performance model (Sec. Methodology: eq. roofline, eq. c-limit; Sec. Algorithm: eq. pr:icop)
# ----------------------------------------------------------------------------------------
def cop_budget(D: int, pi_tflops: float, gamma_tcops: float) -> float:
    """eq. c-limit: the most COPs per score that keep the COP roofline above the
    matrix peak, C <= 2 D gamma / pi."""
    return 2.0 * D * gamma_tcops / pi_tflops


def cop_intensity(D: int, C: float) -> float:
    """eq. pr:icop: FLOPs per COP of the bin-reduce kernel, I_COP = 2D / C."""
    return 2.0 * D / C


def roofline_gflops(pi_tflops: float, beta_gbs: float, gamma_tcops: float, i_mem: float, i_cop: float) -> float:
    """eq. roofline: attainable GFLOP/s = min(pi, beta * I_MEM, gamma * I_COP)."""
    return min(pi_tflops * 1e3, beta_gbs * i_mem, gamma_tcops * 1e3 * i_cop)


# ----------------------------------------------------------------------------------------
# reference quantisers, written from the definitions of the formats
# ----------------------------------------------------------------------------------------
def bf16_round(x):
    """Round FP32 values to the nearest BF16 value, ties to an even BF16 mantissa.

    Candidates are the BF16 value obtained by dropping the low 16 bits (towards zero)
    and its successor away from zero; the nearer one is taken in exact FP64
    arithmetic.  Returns (values as float32, 16-bit codes).
    """
    x = np.ascontiguousarray(x, np.float32)
    u = x.view(np.uint32)
    lo_bits = u & np.uint32(0xFFFF0000)
    hi_bits = lo_bits + np.uint32(0x00010000)
    lo = lo_bits.view(np.float32).astype(np.float64)
    hi = hi_bits.view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo = np.abs(xd - lo)
    dhi = np.abs(hi - xd)
    lo_even = ((lo_bits >> np.uint32(16)) & np.uint32(1)) == 0
    take_hi = (dhi < dlo) | ((dhi == dlo) & ~lo_even)
    bits = np.where(take_hi, hi_bits, lo_bits)
    codes = (bits >> np.uint32(16)).astype(np.uint16)
    return bits.view(np.float32), codes


def fp8_e4m3_table():
    """Non-negative finite values of FP8 E4M3 (OCP, no infinities; code 0x7F is NaN).

    Code c = (E << 3) | m: E = 0 gives m/8 * 2^-6, otherwise (1 + m/8) * 2^(E-7).
    The largest finite value is code 0x7E = 448.
    """
    vals = []
    for c in range(0x7F):
        E, m = c >> 3, c & 7
        vals.append((m / 8.0) * 2.0 ** -6 if E == 0 else (1.0 + m / 8.0) * 2.0 ** (E - 7))
    return np.array(vals, np.float64)


FP8_MAX = 448.0


def fp8_round(y):
    """Round to the nearest E4M3 value (ties to an even code), saturating at +-448.

    Returns (values as float64, 8-bit codes with the sign in bit 7)."""
    y = np.asarray(y, np.float64)
    tab = fp8_e4m3_table()
    a = np.minimum(np.abs(y), FP8_MAX)
    hi = np.clip(np.searchsorted(tab, a, side="left"), 0, len(tab) - 1)
    lo = np.clip(hi - 1, 0, len(tab) - 1)
    dlo = np.abs(a - tab[lo])
    dhi = np.abs(tab[hi] - a)
    take_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    c = np.where(take_hi, hi, lo).astype(np.uint8)
    neg = np.signbit(y)
    codes = c | np.where(neg, np.uint8(0x80), np.uint8(0)).astype(np.uint8)
    vals = np.where(neg, -tab[c], tab[c])
    return vals, codes


def fp8_row_exponent(amax):
    """Smallest integer e with amax <= 448 * 2^e (e = 0 for an all-zero row), clamped to [-127, 127]."""
    amax = np.asarray(amax, np.float64)
    _, E1 = np.frexp(amax)  # amax in [2^(E1-1), 2^E1)
    e = (E1 - 1 - 8).astype(np.int64)
    e = np.where(amax > np.ldexp(FP8_MAX, e), e + 1, e)
    e = np.where(amax == 0, 0, e)
    e = np.clip(e, -127, 127)
    return e


def fp8_quantize_rows(X):
    """Per-row power-of-two scaled E4M3: x ~ code(x * 2^-e) * 2^e.

    Returns (dequantised float32 rows, codes uint8, exponents int64)."""
    X = np.ascontiguousarray(X, np.float32)
    amax = np.abs(X).max(axis=1).astype(np.float64) if X.shape[1] else np.zeros(X.shape[0])
    e = fp8_row_exponent(amax)
    y = X.astype(np.float64) * np.ldexp(1.0, -e)[:, None]
    vals, codes = fp8_round(y)
    deq = (vals * np.ldexp(1.0, e)[:, None]).astype(np.float32)
    return deq, codes, e


def normalize_rows_f32(X):
    """Unit-normalise rows in FP32: |x|^2 summed in increasing dimension order with one
    rounding per product and per sum, a correctly rounded square root and divisions; a
    zero row stays zero."""
    X = np.ascontiguousarray(X, np.float32)
    acc = np.zeros(X.shape[0], np.float32)
    for d in range(X.shape[1]):
        acc = (acc + (X[:, d] * X[:, d]).astype(np.float32)).astype(np.float32)
    nrm = np.sqrt(acc).astype(np.float32)
    safe = np.where(nrm > 0, nrm, np.float32(1)).astype(np.float32)
    out = (X / safe[:, None]).astype(np.float32)
    out[nrm == 0] = 0
    return out


def quantize_like_library(X, metric, compute: str):
    """The input rows as the search computes with them: cosine rows unit-normalised in FP32,
    then rounded to the compute format (fp32: unchanged, bf16: RNE, fp8: per-row E4M3)."""
    X = np.ascontiguousarray(X, np.float32)
    if _metric(metric) == COSINE:
        X = normalize_rows_f32(X)
    if compute == "fp32":
        return X
    if compute == "bf16":
        return bf16_round(X)[0]
    if compute == "fp8":
        return fp8_quantize_rows(X)[0]
    raise ValueError(compute)
