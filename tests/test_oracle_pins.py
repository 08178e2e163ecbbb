"""Pins of the CPU oracle against things other than itself (no GPU needed).

Each test names the passage of the paper it checks and the independent fact that
pins it: brute force, a library routine, an exact enumeration, or an identity.
"""
import itertools
import math
import struct
from fractions import Fraction

import numpy as np
import pytest
import scipy.spatial.distance as ssd

import oracle


# ---------------------------------------------------------------- bins (Algorithm 1)
def test_bins_partition_exhaustive():
    """Contiguous balanced bins: every row in exactly one bin, sizes differ by <= 1,
    and the bin of row j equals floor(((j+1)L - 1)/N) (an independent closed form)."""
    for N in range(1, 90):
        for L in range(1, N + 1):
            starts = [oracle.bin_start(b, N, L) for b in range(L + 1)]
            assert starts[0] == 0 and starts[-1] == N
            sizes = np.diff(starts)
            assert sizes.min() >= 1 and sizes.max() - sizes.min() <= 1
            for j in range(N):
                b = oracle.bin_of(j, N, L)
                assert starts[b] <= j < starts[b + 1]
                assert b == ((j + 1) * L - 1) // N


def test_bins_power_of_two_is_shift_right():
    """With N = L * 2^W the balanced partition is Algorithm 1's ShiftRight(j, W)."""
    for W in range(0, 6):
        for L in (1, 3, 8, 64):
            N = L << W
            for j in range(N):
                assert oracle.bin_of(j, N, L) == j >> W


def _brute_bins(S, L, minimize):
    M, N = S.shape
    V = np.empty((M, L))
    A = np.empty((M, L), np.int64)
    for b in range(L):
        j0, j1 = oracle.bin_start(b, N, L), oracle.bin_start(b + 1, N, L)
        blk = S[:, j0:j1]
        a = np.argmin(blk, axis=1) if minimize else np.argmax(blk, axis=1)  # first occurrence
        V[:, b] = blk[np.arange(M), a]
        A[:, b] = j0 + a
    return V, A


@pytest.mark.parametrize("minimize", [False, True])
def test_partial_reduce_vs_bruteforce_with_ties(minimize):
    """Algorithm 1 (strict compare, increasing j) == per-bin argmax with first-occurrence
    ties, on small-integer scores full of ties, for every L <= N."""
    rng = np.random.default_rng(7)
    for N in range(1, 13):
        S = rng.integers(-3, 4, size=(5, N)).astype(np.float64)
        for L in range(1, N + 1):
            V, A = oracle.partial_reduce(S, L, minimize)
            Vb, Ab = _brute_bins(S, L, minimize)
            np.testing.assert_array_equal(V, Vb)
            np.testing.assert_array_equal(A, Ab)


def test_search_invariants():
    """Winners lie in their bin, equal the bin's true best, ties go to the lowest row;
    the runner-up is the best of the other rows."""
    rng = np.random.default_rng(3)
    Q = rng.integers(-2, 3, size=(6, 4)).astype(np.float32)
    X = rng.integers(-2, 3, size=(50, 4)).astype(np.float32)
    for metric in ("mips", "l2", "cosine"):
        S, _ = oracle.scores(Q, X, metric)
        mn = oracle.minimize_for(metric)
        for L in (1, 2, 7, 16, 50):
            r = oracle.search(Q, X, metric, L, 1, bins=True)
            for i in range(6):
                for b in range(L):
                    j0, j1 = oracle.bin_start(b, 50, L), oracle.bin_start(b + 1, 50, L)
                    a = r["bin_i"][i, b]
                    assert j0 <= a < j1
                    blk = S[i, j0:j1]
                    best = blk.min() if mn else blk.max()
                    assert r["bin_v"][i, b] == best
                    assert a == j0 + int(np.flatnonzero(blk == best)[0])
                    others = np.delete(blk, a - j0)
                    if others.size:
                        assert r["bin2_v"][i, b] == (others.min() if mn else others.max())


# ---------------------------------------------------------------- scores (Sec. 2, appendix)
def test_scores_vs_library():
    """MIPS == numpy's matrix product; cosine == 1 - scipy's cosine distance; zero norm -> 0."""
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((7, 33)).astype(np.float32)
    X = rng.standard_normal((40, 33)).astype(np.float32)
    X[5] = 0
    S, _ = oracle.scores(Q, X, "mips")
    np.testing.assert_allclose(S, Q.astype(np.float64) @ X.astype(np.float64).T, rtol=1e-12, atol=1e-12)
    C, _ = oracle.scores(Q, X, "cosine")
    for i in range(7):
        for j in range(40):
            if j == 5:
                assert C[i, j] == 0.0
            else:
                ref = 1.0 - ssd.cosine(Q[i].astype(np.float64), X[j].astype(np.float64))
                assert abs(C[i, j] - ref) < 1e-12


def test_relaxed_l2_identity_and_ranking():
    """Appendix (eq. l2-suboptimal, eq. l2final): 2*(|x|^2/2 - <q,x>) + |q|^2 = |q - x|^2,
    so ranking by the relaxed score equals ranking by the Euclidean distance (integer data:
    exact in FP64)."""
    rng = np.random.default_rng(2)
    Q = rng.integers(0, 256, size=(9, 16)).astype(np.float32)
    X = rng.integers(0, 256, size=(300, 16)).astype(np.float32)
    S, _ = oracle.scores(Q, X, "l2")
    d2 = ((Q[:, None, :].astype(np.float64) - X[None, :, :].astype(np.float64)) ** 2).sum(-1)
    qq = (Q.astype(np.float64) ** 2).sum(1)[:, None]
    np.testing.assert_array_equal(2 * S + qq, d2)
    for i in range(9):
        o1 = np.lexsort((np.arange(300), S[i]))
        o2 = np.lexsort((np.arange(300), ssd.cdist(Q[i:i + 1], X, "euclidean")[0]))
        np.testing.assert_array_equal(o1, o2)


# ---------------------------------------------------------------- top-K (ExactRescoring)
@pytest.mark.parametrize("metric", ["mips", "l2", "cosine"])
def test_L_equals_N_is_exact_knn(metric):
    """With one row per bin every row is a winner, so the result is the exact K-NN
    (eq. 1 / eq. 2), checked against numpy's stable sort of the FP64 scores."""
    rng = np.random.default_rng(4)
    Q = rng.integers(-3, 4, size=(5, 6)).astype(np.float32)
    X = rng.integers(-3, 4, size=(37, 6)).astype(np.float32)
    S, _ = oracle.scores(Q, X, metric)
    mn = oracle.minimize_for(metric)
    r = oracle.search(Q, X, metric, 37, 9, exact=True)
    for i in range(5):
        key = S[i] if mn else -S[i]
        order = np.lexsort((np.arange(37), key))[:9]
        np.testing.assert_array_equal(r["top_i"][i], order)
        np.testing.assert_array_equal(r["ex_i"][i], order)


def test_K1_exact_for_any_L_and_L1_is_argmax():
    """The global best is always some bin's winner: K = 1 is exact for every L; L = 1, K = 1
    is numpy's argmax (first occurrence)."""
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((4, 8)).astype(np.float32)
    X = rng.standard_normal((200, 8)).astype(np.float32)
    S, _ = oracle.scores(Q, X, "mips")
    for L in (1, 2, 3, 17, 64, 200):
        r = oracle.search(Q, X, "mips", L, 1, exact=True)
        np.testing.assert_array_equal(r["top_i"][:, 0], np.argmax(S, axis=1))
        np.testing.assert_array_equal(r["ex_i"][:, 0], np.argmax(S, axis=1))


def test_nested_bins_recall_monotone():
    """Refining every bin into c pieces (L' = c L, N divisible) can only keep more
    true neighbours: per-query recall is non-decreasing in c."""
    rng = np.random.default_rng(6)
    Q = rng.standard_normal((16, 8)).astype(np.float32)
    X = rng.standard_normal((960, 8)).astype(np.float32)
    prev = None
    for L in (15, 30, 60, 120, 240, 960):
        r = oracle.search(Q, X, "mips", L, 10, exact=True)
        rec = oracle.recall(r["top_i"], r["ex_i"])
        if prev is not None:
            assert np.all(rec >= prev - 1e-12)
        prev = rec
    assert np.all(prev == 1.0)


# ---------------------------------------------------------------- recall model (Sec. 5.1)
def _enumerated_recall(N, L, K):
    """Exact E[recall] by running the oracle on every placement of the K true neighbours."""
    tot = Fraction(0)
    cnt = 0
    Q = np.ones((1, 1), np.float32)
    for P in itertools.combinations(range(N), K):
        x = np.arange(N, dtype=np.float32)[:, None] * 0.0 - np.arange(N, dtype=np.float32)[:, None]
        for rank, p in enumerate(P):
            x[p, 0] = 1000.0 - rank  # the K best rows, all distinct
        r = oracle.search(Q, x, "mips", L, K, exact=True)
        tot += Fraction(len(set(r["top_i"][0]) & set(r["ex_i"][0])), K)
        cnt += 1
    return tot / cnt


@pytest.mark.parametrize("N,L,K,expect", [
    (8, 4, 2, Fraction(13, 14)),
    (12, 4, 3, Fraction(136, 165)),
    (12, 5, 4, Fraction(177, 220)),
    (9, 9, 4, Fraction(1)),
    (10, 3, 3, None),
    (11, 4, 2, None),
])
def test_recall_expectation_by_enumeration(N, L, K, expect):
    """Sec. 5.1: recall = (#bins holding a true neighbour)/K.  The closed form
    (1/K) sum_b [1 - C(N-B_b,K)/C(N,K)] equals exhaustive enumeration of all placements
    through the oracle's own search, and is >= the paper's bound ((L-1)/L)^(K-1)."""
    enum = _enumerated_recall(N, L, K)
    closed = oracle.recall_exact_balanced(N, L, K, exact_fraction=True)
    assert enum == closed
    if expect is not None:
        assert closed == expect
    assert float(closed) >= oracle.recall_bound_paper(K, L) - 1e-15
    assert abs(float(closed) - oracle.recall_exact_balanced(N, L, K)) < 1e-12


def test_recall_monte_carlo_at_mips_small_shape():
    """N = 65536, L = 2048, K = 10 with i.i.d. scores (row order independent of the query):
    the mean recall over 3200 queries lies within 5 sigma of the exact balanced-bin
    expectation and above the paper's bound."""
    N, L, K = 65536, 2048, 10
    exact = oracle.recall_exact_balanced(N, L, K)
    bound = oracle.recall_bound_paper(K, L)
    assert abs(exact - 0.997874) < 1e-6 and abs(bound - 0.995614) < 1e-6
    rng = np.random.default_rng(11)
    recs = []
    for _ in range(50):
        S = rng.standard_normal((64, N))
        V, A = oracle.partial_reduce(S, L, False)
        _, top = oracle.topk_pairs(V, A, K, False)
        truth = np.argsort(-S, axis=1, kind="stable")[:, :K]
        recs.append(oracle.recall(top, truth))
    recs = np.concatenate(recs)
    sigma = recs.std() / math.sqrt(recs.size)
    assert abs(recs.mean() - exact) < 5 * sigma + 1e-12
    assert recs.mean() > bound


def test_exact_expectation_bins_at_the_sift_shape():
    """N = 10^6, K = 10 (the SIFT-shaped workload).  With N much larger than K, drawing the
    neighbours' rows without replacement barely differs from placing them independently,
    so the exact balanced-bin expectation must sit within 1e-4 of the closed form
    L (1 - (1 - 1/L)^K) / K, and above the paper's bound.  L = 176 (eq. l:approx) gives
    0.9748; the smallest L whose exact expectation reaches 0.95 is 88."""
    N, K = 1_000_000, 10
    for L in (87, 88, 176):
        exact = oracle.recall_exact_balanced(N, L, K)
        indep = L * (1.0 - (1.0 - 1.0 / L) ** K) / K
        assert abs(exact - indep) < 1e-4
        assert exact >= oracle.recall_bound_paper(K, L)
    assert abs(oracle.recall_exact_balanced(N, 176, K) - 0.97482) < 1e-5
    assert oracle.recall_exact_balanced(N, 88, K) >= 0.95 > oracle.recall_exact_balanced(N, 87, K)


def test_bins_for_recall():
    """eq. l:approx: K = 10, r = 0.95 -> L >= 1/(1 - 0.95^(1/9)) = 175.97 -> 176; the
    first-order form (K-1)/(1-r) gives 180; the result is the smallest L meeting eq. recall."""
    assert oracle.bins_for_recall(10, 0.95) == 176
    assert abs(oracle.bins_for_recall_approx(10, 0.95) - 180.0) < 1e-9
    for K in (2, 5, 10, 64, 100):
        for r in (0.5, 0.9, 0.95, 0.99):
            L = oracle.bins_for_recall(K, r)
            assert oracle.recall_bound_paper(K, L) >= r
            if L > K:
                assert oracle.recall_bound_paper(K, L - 1) < r
    assert oracle.bins_for_recall(1, 0.99) == 1
    assert oracle.bins_for_recall(10, 0.95, N=100) == 100
    assert oracle.bins_for_recall(64, 0.95) == 1229 and oracle.bins_for_recall(100, 0.95) == 1931


# ---------------------------------------------------------------- quantisers
def test_bf16_round_vs_torch():
    """RNE to BF16 == torch's float32 -> bfloat16 conversion (a library routine)."""
    import torch
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(200000).astype(np.float32) * 100,
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 255.0, 256.0, 257.0, -3e-39],
                                 np.float32)])
    mid = (np.arange(1, 4096, dtype=np.uint32) << 16 | np.uint32(0x8000)) + np.uint32(0x3F800000)
    x = np.concatenate([x, mid.view(np.float32)])  # exact ties
    v, codes = oracle.bf16_round(x)
    t = torch.from_numpy(x).to(torch.bfloat16)
    np.testing.assert_array_equal(codes, t.view(torch.int16).numpy().view(np.uint16))
    np.testing.assert_array_equal(v, t.float().numpy())
    ints = np.arange(0, 256, dtype=np.float32)
    np.testing.assert_array_equal(oracle.bf16_round(ints)[0], ints)  # 0..255 exact in BF16


def test_fp8_table_and_round_vs_torch():
    """E4M3 (OCP): 127 non-negative finite values, max 448, min subnormal 2^-9, min normal
    2^-6; RNE agrees with torch's float8_e4m3fn conversion on in-range values; saturation."""
    import torch
    tab = oracle.fp8_e4m3_table()
    assert tab.size == 127 and tab[-1] == 448.0 and tab[1] == 2.0 ** -9 and tab[8] == 2.0 ** -6
    assert np.all(np.diff(tab) > 0)
    rng = np.random.default_rng(9)
    y = np.concatenate([rng.uniform(-448, 448, 100000), rng.standard_normal(100000) * 0.01,
                        (tab[:-1] + tab[1:]) / 2, -(tab[:-1] + tab[1:]) / 2, tab, -tab])
    y = y.astype(np.float32).astype(np.float64)
    vals, codes = oracle.fp8_round(y)
    t = torch.from_numpy(y.astype(np.float32)).to(torch.float8_e4m3fn)
    np.testing.assert_array_equal(codes, t.view(torch.uint8).numpy())
    np.testing.assert_array_equal(vals, t.float().numpy().astype(np.float64))
    v2, c2 = oracle.fp8_round(np.array([500.0, -1e6, 449.0]))
    assert list(v2) == [448.0, -448.0, 448.0] and list(c2) == [0x7E, 0xFE, 0x7E]


def test_fp8_row_exponent_minimal():
    """The row exponent is the smallest e with amax <= 448 * 2^e."""
    rng = np.random.default_rng(10)
    amax = np.abs(rng.standard_normal(5000)) * 10.0 ** rng.uniform(-8, 8, 5000)
    amax = np.concatenate([amax, [448.0, 448.0 * 2 ** -3, 449.0, 1.0, 0.0]])
    e = oracle.fp8_row_exponent(amax)
    nz = amax > 0
    assert np.all(amax[nz] <= 448.0 * 2.0 ** e[nz])
    assert np.all(amax[nz] > 448.0 * 2.0 ** (e[nz] - 1))
    assert e[-1] == 0 and e[-5] == 0 and e[-3] == 1 and e[-2] == -8


def _f32(v: float) -> float:
    """Round a Python float (FP64) to the nearest FP32 value, ties to even."""
    return struct.unpack("<f", struct.pack("<f", v))[0]


def _normalize_row_scalar(row):
    """One row unit-normalised with scalar FP32 steps, written independently of the
    oracle: Python FP64 arithmetic with a rounding to FP32 after every product, sum,
    square root and division.  (Each of these FP64 results rounded once more to FP32
    is the correctly rounded FP32 result: FP64 carries more than 2 * 24 + 2 bits.)"""
    acc = 0.0
    for v in row:
        acc = _f32(acc + _f32(float(v) * float(v)))
    nrm = _f32(math.sqrt(acc))
    if nrm == 0.0:
        return [0.0] * len(row)
    return [_f32(float(v) / nrm) for v in row]


def test_normalize_rows_f32_bit_exact_vs_scalar_loop():
    """Cosine preparation (Sec. 2, cosine similarity as MIPS on normalised rows): the
    oracle's vectorised FP32 normalisation equals, bit for bit, a scalar loop that rounds
    to FP32 after every operation in increasing dimension order, on rows of ordinary,
    tiny, huge and mixed magnitudes, single-entry rows and a zero row; and every
    non-zero result has unit FP64 norm within the FP32 rounding of D + 2 steps."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((64, 100)).astype(np.float32)
    X[3] = 0
    X[4] = 0
    X[4, 17] = -3.5
    X[5] *= np.float32(1e-18)
    X[6] *= np.float32(1e17)
    X[7] = (rng.standard_normal(100) * 10.0 ** rng.uniform(-6, 6, 100)).astype(np.float32)
    X[8, :50] = 1.0
    Xn = oracle.normalize_rows_f32(X)
    ref = np.array([_normalize_row_scalar(r) for r in X], np.float32)
    np.testing.assert_array_equal(Xn.view(np.uint32), ref.view(np.uint32))
    n = np.sqrt((Xn.astype(np.float64) ** 2).sum(1))
    nz = np.abs(X).max(1) > 0
    assert np.all(np.abs(n[nz] - 1) < (100 + 2) * 2.0 ** -24 * 2) and np.all(n[~nz] == 0)


# ---------------------------------------------------------------- rounding magnitudes
def _emulated_f32_scores(Q, X, metric, order):
    """FP32 evaluation of the scores the way a matrix unit may sum them: products rounded
    to FP32, then summed in FP32 in the given order of dimensions ("seq", "rev" or
    "pairs"); L2 starts from -|x|^2/2 summed in FP32; cosine normalises both sides in
    FP32 first.  Returns an M x N FP64 array holding the FP32 results."""
    Q = np.asarray(Q, np.float32)
    X = np.asarray(X, np.float32)
    if metric == "cosine":
        Q, X = oracle.normalize_rows_f32(Q), oracle.normalize_rows_f32(X)
    P = Q[:, None, :] * X[None, :, :]  # FP32 products, correctly rounded
    D = P.shape[2]
    if metric == "l2":
        h = np.zeros(X.shape[0], np.float32)
        for d in range(D):
            h = h + X[:, d] * X[:, d]
        acc = np.broadcast_to(-(h * np.float32(0.5)), P.shape[:2]).astype(np.float32)
    else:
        acc = np.zeros(P.shape[:2], np.float32)
    if order == "pairs":
        T = P
        while T.shape[2] > 1:
            if T.shape[2] % 2:
                T = np.concatenate([T, np.zeros(T.shape[:2] + (1,), np.float32)], axis=2)
            T = T[:, :, 0::2] + T[:, :, 1::2]
        acc = acc + T[:, :, 0]
    else:
        for d in (range(D) if order == "seq" else range(D - 1, -1, -1)):
            acc = acc + P[:, :, d]
    s = acc.astype(np.float64)
    return -s if metric == "l2" else s  # the accumulator holds <q,x> - |x|^2/2


def _gamma(n, u=2.0 ** -24):
    return n * u / (1 - n * u)


@pytest.mark.parametrize("metric", ["mips", "l2", "cosine"])
def test_magnitudes_bound_fp32_rounding(metric):
    """The parity rule's rounding bound e = gamma_n * mag with n = D + 3 (Higham's bound
    for a sum of products in any order) holds for FP32 evaluations of the score in three
    summation orders, at the round-to-nearest unit 2^-24 (the tests use twice that).  For
    L2 the data make the rounding of |x|^2/2 dominate: the error is far above
    gamma_n * sum|q_k x_k|, so a magnitude without the 1/2 |x|^2 term fails here."""
    rng = np.random.default_rng(21)
    D = 96
    if metric == "l2":
        Q = (rng.standard_normal((24, D)) * 1e-3).astype(np.float32)
        X = (rng.standard_normal((200, D)) * 100.0).astype(np.float32)
    else:
        Q = rng.standard_normal((24, D)).astype(np.float32)
        X = (rng.standard_normal((200, D)) * np.exp(rng.uniform(-2, 2, (200, 1)))).astype(np.float32)
    S, MAG = oracle.scores(Q, X, metric)
    g = _gamma(D + 3)
    worst = 0.0
    for order in ("seq", "rev", "pairs"):
        err = np.abs(_emulated_f32_scores(Q, X, metric, order) - S)
        assert np.all(err <= g * MAG), (order, float(np.max(err / (g * MAG))))
        worst = max(worst, float(np.max(err / (g * MAG))))
    assert worst > 1e-3  # the comparison is not vacuous
    if metric == "l2":
        dot_mag = np.abs(Q.astype(np.float64)) @ np.abs(X.astype(np.float64)).T
        err = np.abs(_emulated_f32_scores(Q, X, metric, "seq") - S)
        assert np.max(err / (g * dot_mag)) > 10.0


def test_magnitudes_equality_cases_and_invariances():
    """Magnitudes: never below |score| (MIPS, L2) or |score| + 1 (cosine); equal to them
    when no cancellation can occur (MIPS and cosine on non-negative data, L2 with
    non-positive queries against non-negative rows, L2 with a zero query: 1/2 |x|^2);
    unchanged when a query changes sign; MIPS magnitudes scale with the query; cosine
    magnitudes are scale-free; a zero-norm cosine pair has score 0 and magnitude 1."""
    rng = np.random.default_rng(22)
    Qp = rng.integers(0, 9, (5, 12)).astype(np.float32)
    Xp = rng.integers(0, 9, (30, 12)).astype(np.float32)
    Qp[0, 0] = 1.0
    Xp[:, 1] = 1.0  # no zero rows
    Qp[:, 1] = 1.0
    Qr = rng.standard_normal((5, 12)).astype(np.float32)
    Xr = rng.standard_normal((30, 12)).astype(np.float32)
    for metric in ("mips", "l2", "cosine"):
        S, MAG = oracle.scores(Qr, Xr, metric)
        extra = 1.0 if metric == "cosine" else 0.0
        assert np.all(MAG >= np.abs(S) + extra - 1e-12)
        S2, MAG2 = oracle.scores(-Qr, Xr, metric)
        np.testing.assert_allclose(MAG2, MAG, rtol=1e-14)
    S, MAG = oracle.scores(Qp, Xp, "mips")
    np.testing.assert_array_equal(MAG, S)
    S, MAG = oracle.scores(-Qp, Xp, "l2")
    np.testing.assert_array_equal(MAG, S)
    S, MAG = oracle.scores(np.zeros_like(Qp), Xp, "l2")
    np.testing.assert_array_equal(MAG, S)
    np.testing.assert_array_equal(S, 0.5 * (Xp.astype(np.float64) ** 2).sum(1)[None, :].repeat(5, 0))
    S, MAG = oracle.scores(Qp, Xp, "cosine")
    np.testing.assert_allclose(MAG, S + 1.0, rtol=1e-14)
    _, M1 = oracle.scores(Qr, Xr, "mips")
    _, M4 = oracle.scores(Qr * np.float32(4), Xr, "mips")
    np.testing.assert_array_equal(M4, 4 * M1)
    _, C1 = oracle.scores(Qr, Xr, "cosine")
    _, C2 = oracle.scores(Qr * np.float32(4), Xr * np.float32(0.5), "cosine")
    np.testing.assert_allclose(C2, C1, rtol=1e-14)
    Xz = Xr.copy()
    Xz[7] = 0
    S, MAG = oracle.scores(Qr, Xz, "cosine")
    assert np.all(S[:, 7] == 0.0) and np.all(MAG[:, 7] == 1.0)


@pytest.mark.parametrize("metric", ["mips", "l2", "cosine"])
def test_bin_magnitudes_vs_bruteforce(metric):
    """Per bin the search reports the winner's magnitude (bin_mag) and, over the bin's
    other rows, the best score (bin2_v) and the largest magnitude (bin2_mag), against a
    brute-force scan of the full score and magnitude matrices on tie-rich inputs, for
    every bin count; a bin of one row has no other rows (worst score, magnitude 0)."""
    rng = np.random.default_rng(23)
    Q = rng.integers(-2, 3, size=(4, 5)).astype(np.float32)
    X = rng.integers(-2, 3, size=(23, 5)).astype(np.float32)
    S, MAG = oracle.scores(Q, X, metric)
    mn = oracle.minimize_for(metric)
    worst_v = np.inf if mn else -np.inf
    for L in range(1, 24):
        r = oracle.search(Q, X, metric, L, 1, bins=True)
        for i in range(4):
            for b in range(L):
                j0, j1 = oracle.bin_start(b, 23, L), oracle.bin_start(b + 1, 23, L)
                a = r["bin_i"][i, b]
                assert r["bin_mag"][i, b] == MAG[i, a]
                others = [j for j in range(j0, j1) if j != a]
                if others:
                    sv = S[i, others]
                    assert r["bin2_v"][i, b] == (sv.min() if mn else sv.max())
                    assert r["bin2_mag"][i, b] == MAG[i, others].max()
                else:
                    assert r["bin2_v"][i, b] == worst_v and r["bin2_mag"][i, b] == 0.0


# ---------------------------------------------------------------- tie-aware recall (eq. recall-def)
def _recall_by_enumeration(scores, S, K, minimize):
    """Best overlap of the retrieved rows S with any exact K-NN set: every K-subset T of
    the rows none of whose members is beaten by a row outside it."""
    n = len(scores)
    best = 0
    for T in itertools.combinations(range(n), K):
        inside = [scores[j] for j in T]
        outside = [scores[j] for j in range(n) if j not in T]
        if outside and (max(inside) > min(outside) if minimize else min(inside) < max(outside)):
            continue
        best = max(best, len(set(T) & set(S)))
    return Fraction(best, K)


def _exact_topk_scores(scores, K, minimize):
    return sorted(scores, reverse=not minimize)[:K]


@pytest.mark.parametrize("scores,K,S,minimize,expect", [
    ([6, 5, 5, 5], 2, [1, 2], False, Fraction(1, 2)),   # two tied rows cannot replace the strictly better one
    ([6, 5, 5, 5], 2, [0, 3], False, Fraction(1)),      # any one of the tied rows completes the set
    ([1, 2, 2, 2], 2, [1, 2], True, Fraction(1, 2)),    # the same, minimising
    ([1, 2, 2, 2], 2, [3, 0], True, Fraction(1)),
    ([4, 3, 2, 1], 2, [0, 2], False, Fraction(1, 2)),   # no ties: strict recall
    ([7, 7, 7], 2, [2, 0], False, Fraction(1)),         # all tied: every set is exact
    ([3, 9, 9, 1, 9], 3, [1, 3, 4], False, Fraction(2, 3)),
    ([3, 9, 9, 1, 9], 1, [0], False, Fraction(0)),
])
def test_recall_tie_aware_hand_worked(scores, K, S, minimize, expect):
    """Hand-worked cases of recall with ties in both directions, and the enumeration
    agrees with them."""
    ex = np.array([_exact_topk_scores(scores, K, minimize)], np.float64)
    rs = np.array([[scores[j] for j in S]], np.float64)
    got = oracle.recall_tie_aware(rs, ex, minimize)[0]
    assert got == float(expect)
    assert _recall_by_enumeration(scores, S, K, minimize) == expect


@pytest.mark.parametrize("minimize", [False, True])
def test_recall_tie_aware_vs_enumeration(minimize):
    """The closed form (strictly better retrieved rows + the tied ones that fit) equals the
    best overlap with any exact K-NN set, by enumeration, on small-integer scores full of
    ties, for every K and many retrieved sets; without ties it is the strict recall."""
    rng = np.random.default_rng(24)
    for n in range(1, 9):
        for trial in range(12):
            scores = rng.integers(0, 4, n).tolist()
            for K in range(1, n + 1):
                ex = np.array([_exact_topk_scores(scores, K, minimize)], np.float64)
                for _ in range(4):
                    S = rng.choice(n, K, replace=False).tolist()
                    rs = np.array([[scores[j] for j in S]], np.float64)
                    got = oracle.recall_tie_aware(rs, ex, minimize)[0]
                    assert got == float(_recall_by_enumeration(scores, S, K, minimize)), (scores, K, S)
    scores = rng.permutation(50).astype(np.float64)
    truth = np.argsort(scores if minimize else -scores)[:7]
    for _ in range(20):
        S = rng.choice(50, 7, replace=False)
        got = oracle.recall_tie_aware(scores[S][None], scores[truth][None], minimize)[0]
        assert got == oracle.recall(S[None], truth[None])[0]


# ---------------------------------------------------------------- backward reference
@pytest.mark.parametrize("metric", ["mips", "l2", "cosine"])
def test_backward_vs_finite_differences(metric):
    """Dense FP64 gradient of a softmax cross-entropy over the retrieved scores (selection
    frozen) against central finite differences, at Q = 8, N = 4096, D = 16, K = 64, L = 1024."""
    from paper_2206_14286_amd import datagen
    M, N, D, K, L = 8, 4096, 16, 64, 1024
    Q = datagen.normal(M, D, 101)
    X = datagen.normal(N, D, 100)
    t = datagen.targets(M, K, 102)
    r = oracle.search(Q, X, metric, L, K)
    a = r["top_i"]

    def loss(Qm, Xm):
        s, _ = oracle.pair_scores(Qm, Xm, metric, np.repeat(np.arange(M), K), a.ravel())
        s = s.reshape(M, K)
        z = s - s.max(1, keepdims=True)
        lse = np.log(np.exp(z).sum(1))
        return float(np.mean(lse - z[np.arange(M), t]))

    s, _ = oracle.pair_scores(Q, X, metric, np.repeat(np.arange(M), K), a.ravel())
    s = s.reshape(M, K)
    p = np.exp(s - s.max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    g = p.copy()
    g[np.arange(M), t] -= 1.0
    g /= M
    dQ, dX = oracle.backward(g, a, Q, X, metric)
    h = 1e-3  # FP32 inputs: perturb in FP64 through a float64 copy
    Qd, Xd = Q.astype(np.float64), X.astype(np.float64)
    rng = np.random.default_rng(0)
    coords = [("q", i, d) for i in range(M) for d in range(D)]
    rows = np.unique(a.ravel())
    coords += [("x", int(j), int(d)) for j in rng.choice(rows, 40, replace=False) for d in rng.choice(D, 3)]
    coords += [("x", int(j), 0) for j in np.setdiff1d(np.arange(N), rows)[:5]]

    def loss64(Qm, Xm):
        return loss_fd(Qm, Xm)

    def loss_fd(Qm, Xm):
        qi = np.repeat(np.arange(M), K)
        xj = a.ravel()
        qv, xv = Qm[qi], Xm[xj]
        dot = (qv * xv).sum(1)
        if metric == "mips":
            s = dot
        elif metric == "l2":
            s = 0.5 * (xv * xv).sum(1) - dot
        else:
            s = dot / np.sqrt((qv * qv).sum(1) * (xv * xv).sum(1))
        s = s.reshape(M, K)
        z = s - s.max(1, keepdims=True)
        return float(np.mean(np.log(np.exp(z).sum(1)) - z[np.arange(M), t]))

    assert abs(loss_fd(Qd, Xd) - loss(Q, X)) < 1e-9
    for kind, i, d in coords:
        A_ = Qd if kind == "q" else Xd
        old = A_[i, d]
        A_[i, d] = old + h
        lp = loss64(Qd, Xd)
        A_[i, d] = old - h
        lm = loss64(Qd, Xd)
        A_[i, d] = old
        fd = (lp - lm) / (2 * h)
        an = dQ[i, d] if kind == "q" else dX[i, d]
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an), (kind, i, d, fd, an)
