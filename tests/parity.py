"""Comparison of HIP-path outputs with the FP64 oracle (the parity rule).

Rounding bound for one score summed in FP32 in any order (Higham's inner-product
bound): e = gamma_n * mag, gamma_n = n u / (1 - n u), n = Dpad + 3, with u = 2^-23
(twice the unit roundoff of round-to-nearest, to cover matrix-unit adders that
may truncate) and mag = sum_k |q_k x_k| (+ |x|^2/2 for L2, + 1 for cosine).

  * bins: where the FP64 gap between a bin's winner and the best of its other rows
    exceeds e_w + e_r (e_r from the largest magnitude among the other rows, so the
    winner is then ahead of every other row by more than the bound of the pair) the
    GPU row must equal the oracle's; otherwise any row of the bin whose FP64 score is
    within e_w + e_r of the winner is accepted;
  * values: |V_gpu - s64(row)| <= max(1e-5 |s64|, e(row)), s64 the FP64 score of
    the row the GPU returned;
  * top-K: every row the oracle ranks better than its K-th value by more than
    the bound must be returned, every returned row must be within the bound of
    the oracle's K-th value or better, and values are sorted best first.
"""
import numpy as np

import oracle

# Unit roundoff of the FP8 parity bound: the block-scaled FP8 matrix instruction sums
# its 64-deep products less exactly than FP32 accumulation; its measured error reaches
# 5.4 x gamma_n(2^-23) * mag at depth 64 (test_gpu_boundary.py characterises it over
# 4.2 M dot products), and 8 x 2^-23 is the smallest power of two above that.
FP8_U = 2.0 ** -20


def gamma(dpad: int, u: float = 2.0 ** -23) -> float:
    n = dpad + 3
    return n * u / (1 - n * u)


def check_bins(Q, X, metric, L, gpu_v, gpu_i, ora, dpad, u=2.0 ** -23, value_rtol=1e-5):
    """Returns (n_exact_checked, n_near_tie) and raises AssertionError on a violation."""
    M = Q.shape[0]
    N = X.shape[0]
    g = gamma(dpad, u)
    mn = oracle.minimize_for(metric)
    gv = np.asarray(gpu_v, np.float64)
    gi = np.asarray(gpu_i, np.int64)
    assert gv.shape == (M, L) and gi.shape == (M, L)
    starts = np.array([oracle.bin_start(b, N, L) for b in range(L + 1)])
    # every GPU row must lie in its bin
    assert np.all(gi >= starts[None, :-1]) and np.all(gi < starts[None, 1:]), "row outside its bin"
    tol = g * (ora["bin_mag"] + ora["bin2_mag"]) + 1e-300
    gap = np.abs(ora["bin_v"] - ora["bin2_v"])
    sep = gap > tol
    # separated bins: exact index equality
    bad = sep & (gi != ora["bin_i"])
    if bad.any():
        i, b = np.argwhere(bad)[0]
        raise AssertionError(f"bin ({i},{b}): gpu row {gi[i, b]} != oracle row {ora['bin_i'][i, b]} "
                             f"(gap {gap[i, b]:.3e} > tol {tol[i, b]:.3e})")
    qi = np.repeat(np.arange(M), L)
    s64, mag = oracle.pair_scores(Q, X, metric, qi, gi.ravel())
    s64 = s64.reshape(M, L)
    mag = mag.reshape(M, L)
    # near ties: the returned row must be within the bound of the winner
    worse = (s64 - ora["bin_v"]) if mn else (ora["bin_v"] - s64)
    lim = g * (ora["bin_mag"] + mag)
    assert np.all(worse <= lim + tol), "near-tie row too far from the bin winner"
    err = np.abs(gv - s64)
    lim_v = np.maximum(value_rtol * np.abs(s64), g * mag)
    ratio = float(np.max(err / (gamma(dpad) * mag + 1e-300)))  # error in units of the FP32 bound
    print(f"  bins: max |err| / (gamma_fp32 * mag) = {ratio:.3f}", flush=True)
    if not np.all(err <= lim_v):
        i, b = np.argwhere(err > lim_v)[0]
        raise AssertionError(f"bin value ({i},{b}): gpu {gv[i, b]!r} vs fp64 {s64[i, b]!r} (ratio {ratio:.2f})")
    return int(sep.sum()), int((~sep).sum())


def check_topk(Q, X, metric, K, gpu_v, gpu_i, ora, dpad, u=2.0 ** -23, value_rtol=1e-5, candidates=None):
    """Top-K of the bin winners.  ``candidates``: oracle (values, magnitudes) of the
    candidate set the top-K was taken from (default: the oracle's bin winners)."""
    M = Q.shape[0]
    g = gamma(dpad, u)
    mn = oracle.minimize_for(metric)
    gv = np.asarray(gpu_v, np.float64)
    gi = np.asarray(gpu_i, np.int64)
    bv = ora["bin_v"]
    bm = ora["bin_mag"]
    qi = np.repeat(np.arange(M), K)
    s64, mag = oracle.pair_scores(Q, X, metric, qi, gi.ravel())
    s64 = s64.reshape(M, K)
    mag = mag.reshape(M, K)
    err = np.abs(gv - s64)
    assert np.all(err <= np.maximum(value_rtol * np.abs(s64), g * mag)), "top-K value error"
    # sorted best first
    d = np.diff(gv, axis=1)
    assert np.all(d >= 0) if mn else np.all(d <= 0), "top-K not sorted"
    for i in range(M):
        order = np.lexsort((np.arange(bv.shape[1]), bv[i] if mn else -bv[i]))
        kth = bv[i, order[K - 1]]
        kth_mag = bm[i, order[K - 1]]
        for r in range(K):
            b = order[r]
            t = g * (bm[i, b] + kth_mag) * 2
            clearly_in = (kth - bv[i, b] > t) if mn else (bv[i, b] - kth > t)
            if clearly_in:
                assert ora["bin_i"][i, b] in set(gi[i].tolist()), f"query {i}: missing row {ora['bin_i'][i, b]}"
        for r in range(K):
            t = g * (mag[i, r] + kth_mag) * 2
            ok = (s64[i, r] <= kth + t) if mn else (s64[i, r] >= kth - t)
            assert ok, f"query {i}: returned row {gi[i, r]} is worse than the K-th by more than the bound"
    assert all(len(set(row.tolist())) == K for row in gi), "duplicate rows in a top-K"


def check_rerank(Q, X, metric, compute, K, L, Kr, vals, idx, dpad, u):
    """Rerank parity against the oracle's definition: the top-Kr bin winners of the
    quantised search, rescored in FP64 from the original rows, best K kept.  For every
    query, under the rounding bounds of both stages:
      * every returned value is the FP32 score of its row, best first;
      * every returned row could be a candidate: its quantised score is within the
        bound of its bin's winner, and that bin is not clearly outside the top Kr;
      * every sure candidate (a clear winner of a bin clearly inside the top Kr) whose
        FP64 score clearly beats the K-th returned score is returned.
    Q, X: the caller's rows (float32); vals, idx: the GPU's M x K output.  Returns the
    number of sure rows checked."""
    M, D = Q.shape
    N = X.shape[0]
    vals = np.asarray(vals, np.float64)
    idx = np.asarray(idx, np.int64)
    mn = oracle.minimize_for(metric)
    sign = 1.0 if mn else -1.0  # ascending sign*value = better first
    qi = np.repeat(np.arange(M), K)
    # returned values: FP32 scores of the returned rows, sorted best first
    s64, mag = oracle.pair_scores(Q, X, metric, qi, idx.ravel())
    s64, mag = s64.reshape(M, K), mag.reshape(M, K)
    g32 = gamma(D)
    tol32 = np.maximum(1e-5 * np.abs(s64), g32 * mag) + 1e-30
    np.testing.assert_array_less(np.abs(vals - s64), tol32)
    assert np.all(np.diff(sign * vals, axis=1) >= 0), "rerank output not sorted best first"
    assert all(len(set(row.tolist())) == K for row in idx), "duplicate rows in a top-K"
    # quantised search of the oracle: bins and their winners
    Qq = oracle.quantize_like_library(Q, metric, compute)
    Xq = oracle.quantize_like_library(X, metric, compute)
    mo = "mips" if metric == "cosine" else metric
    ora = oracle.search(Qq, Xq, mo, L, Kr, bins=True)
    gq = gamma(dpad, u)
    starts = np.array([oracle.bin_start(b, N, L) for b in range(L + 1)])
    sq, mq = oracle.pair_scores(Qq, Xq, mo, qi, idx.ravel())
    sq, mq = sq.reshape(M, K), mq.reshape(M, K)
    n_sure_checked = 0
    for i in range(M):
        bv, bm = ora["bin_v"][i], ora["bin_mag"][i]
        order = np.lexsort((np.arange(L), sign * bv))
        kth, k1 = order[Kr - 1], order[Kr] if Kr < L else order[Kr - 1]
        # returned rows are possible candidates
        b = np.searchsorted(starts, idx[i], side="right") - 1
        worse_than_winner = sign * (sq[i] - bv[b])
        assert np.all(worse_than_winner <= gq * (mq[i] + bm[b]) + 1e-30), f"query {i}: a row that cannot win its bin"
        outside = sign * (bv[b] - bv[kth])
        assert np.all(outside <= gq * (bm[b] + bm[kth]) + 1e-30), f"query {i}: a bin outside the top Kr"
        # sure candidates that clearly beat the K-th returned score must be returned
        clear_in = sign * (bv[k1] - bv) > gq * (bm + bm[k1]) if Kr < L else np.ones(L, bool)
        clear_win = np.abs(bv - ora["bin2_v"][i]) > gq * (bm + ora["bin2_mag"][i])
        sure = ora["bin_i"][i][clear_in & clear_win]
        if sure.size == 0:
            continue
        cs, cm = oracle.pair_scores(Q, X, metric, np.full(sure.size, i), sure)
        beats = sign * (s64[i, K - 1] - cs) > g32 * (cm + mag[i, K - 1]) + 1e-5 * np.abs(cs)
        must = set(sure[beats].tolist())
        n_sure_checked += len(must)
        assert must <= set(idx[i].tolist()), f"query {i}: missing rows {sorted(must - set(idx[i].tolist()))}"
    return n_sure_checked
