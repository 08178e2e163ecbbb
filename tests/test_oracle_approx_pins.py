"""Pins of the oracle's approx_max_k op on a given score matrix (App. A.1; Sec. 5,
Algorithm 1 and ExactRescoring), each against something other than the oracle itself:
a textbook sort, numpy's argmax, a plain per-bin scan, the transpose identity, and the
sharding property of the input-size override."""
import numpy as np
import pytest

import oracle


def _ints(rng, shape, lo=-3, hi=4):
    return rng.integers(lo, hi, size=shape).astype(np.float64)


def _scan_bins(s, L, minimize):
    """Per bin, walk the slice upwards and keep a strictly better score (plain loops)."""
    n = len(s)
    V, A = [], []
    for b in range(L):
        j0, j1 = (b * n) // L, ((b + 1) * n) // L
        bv, bj = s[j0], j0
        for j in range(j0 + 1, j1):
            if (s[j] < bv) if minimize else (s[j] > bv):
                bv, bj = s[j], j
        V.append(bv)
        A.append(bj)
    return np.array(V), np.array(A)


@pytest.mark.parametrize("minimize", [False, True])
def test_bins_match_plain_scan_both_dims(minimize):
    rng = np.random.default_rng(11)
    for n in (1, 2, 5, 9, 16, 23):
        S = _ints(rng, (4, n))
        for L in sorted({1, min(2, n), n // 3 or 1, n - 1 or 1, n}):
            V, A = oracle.approx_top_k(S, 1, L, dim=1, minimize=minimize, aggregate=False)
            Vt, At = oracle.approx_top_k(S.T.copy(), 1, L, dim=0, minimize=minimize, aggregate=False)
            for i in range(4):
                sv, sa = _scan_bins(S[i], L, minimize)
                np.testing.assert_array_equal(V[i], sv)
                np.testing.assert_array_equal(A[i], sa)
                np.testing.assert_array_equal(Vt[:, i], sv)
                np.testing.assert_array_equal(At[:, i], sa)


def test_signed_zeros_and_masked_scores():
    """-0 and +0 tie (the strict comparison sees them equal), and a bin of -inf scores
    reports its first position."""
    S = np.array([[-0.0, 0.0, -0.0, 0.0, -np.inf, -np.inf, -np.inf, 1.0],
                  [0.0, -0.0, 0.0, -0.0, -np.inf, -np.inf, -np.inf, -np.inf]])
    V, A = oracle.approx_top_k(S, 1, 2, aggregate=False)
    np.testing.assert_array_equal(A, [[0, 7], [0, 4]])
    for i in range(2):
        np.testing.assert_array_equal(A[i], _scan_bins(S[i], 2, False)[1])
    _, A = oracle.approx_top_k(S, 2, 8)
    np.testing.assert_array_equal(A, [[7, 0], [0, 1]])


@pytest.mark.parametrize("minimize", [False, True])
def test_L_equals_n_is_textbook_topk(minimize):
    """One score per bin: every score is a winner, so the op returns the K best of the
    slice ordered (better first, lower index first), as Python's sorted() gives."""
    rng = np.random.default_rng(12)
    S = _ints(rng, (6, 40))
    for K in (1, 5, 40):
        V, A = oracle.approx_top_k(S, K, 40, minimize=minimize)
        for i in range(6):
            order = sorted(range(40), key=lambda j: ((S[i, j] if minimize else -S[i, j]), j))[:K]
            np.testing.assert_array_equal(A[i], order)
            np.testing.assert_array_equal(V[i], S[i, order])


def test_K1_is_argmax_for_any_L():
    """The slice's best score is always a bin winner: K = 1 gives numpy's argmax
    (first occurrence) for every L."""
    rng = np.random.default_rng(13)
    S = _ints(rng, (8, 300), -20, 21)
    for L in (1, 2, 7, 64, 299, 300):
        _, A = oracle.approx_top_k(S, 1, L)
        np.testing.assert_array_equal(A[:, 0], np.argmax(S, axis=1))
        _, A = oracle.approx_top_k(S, 1, L, minimize=True)
        np.testing.assert_array_equal(A[:, 0], np.argmin(S, axis=1))


def test_reduction_dim0_is_the_transpose():
    rng = np.random.default_rng(14)
    S = rng.standard_normal((57, 13))
    for agg in (True, False):
        V1, A1 = oracle.approx_top_k(S, 4, 9, dim=0, aggregate=agg)
        V2, A2 = oracle.approx_top_k(S.T.copy(), 4, 9, dim=1, aggregate=agg)
        np.testing.assert_array_equal(V1, V2.T)
        np.testing.assert_array_equal(A1, A2.T)
        assert V1.shape == ((4 if agg else 9), 13)


def test_bins_from_recall_target():
    """Without an override the op uses eq. l:approx's exact inverse (K = 10, r = 0.95 -> 176),
    clamped to the slice length."""
    assert oracle.approx_bins(1_000_000, 10) == 176
    assert oracle.approx_bins(100, 10) == 100
    assert oracle.approx_bins(50, 1) == 1
    assert oracle.approx_bins(7, 7) == 7


def test_override_gives_shards_the_global_bins():
    """A slice cut into G bin-aligned shards, each reduced with the override set to the
    whole length: the shards' bins, side by side, are the whole slice's bins, and the
    top-K of the shards' top-Ks is the whole slice's top-K (the distributed use of the
    option)."""
    rng = np.random.default_rng(15)
    G, n_sh, K = 4, 2816, 10
    n = G * n_sh
    L_all = oracle.approx_bins(n, K)
    L_sh = oracle.approx_bins(n_sh, K, 0.95, n)
    assert L_all == 176 and L_sh * G == L_all
    S = rng.standard_normal((5, n))
    Vg, Ag = oracle.approx_top_k(S, K, L_all, aggregate=False)
    parts_v, parts_a, top_v, top_a = [], [], [], []
    for g in range(G):
        blk = S[:, g * n_sh:(g + 1) * n_sh]
        v, a = oracle.approx_top_k(blk, K, L_sh, aggregate=False)
        parts_v.append(v)
        parts_a.append(a + g * n_sh)
        v, a = oracle.approx_top_k(blk, K, L_sh)
        top_v.append(v)
        top_a.append(a + g * n_sh)
    np.testing.assert_array_equal(np.concatenate(parts_v, 1), Vg)
    np.testing.assert_array_equal(np.concatenate(parts_a, 1), Ag)
    Vt, At = oracle.approx_top_k(S, K, L_all)
    cv, ca = np.concatenate(top_v, 1), np.concatenate(top_a, 1)
    for i in range(5):
        order = np.lexsort((ca[i], -cv[i]))[:K]
        np.testing.assert_array_equal(ca[i, order], At[i])
        np.testing.assert_array_equal(cv[i, order], Vt[i])
