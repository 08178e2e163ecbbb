"""GPU parity of the approx_max_k op on a given score matrix (``knn_approx_top_k``)
against the oracle: no arithmetic is done on the scores, so values and indices must
match bit for bit (run on an MI355X)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2206_14286_amd import datagen, knn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(rows, cols, kind, dtype, pad, seed):
    """(device tensor with row stride cols + pad, the same values as float64 on the host)."""
    a = datagen.score_matrix(rows, cols + pad, seed, kind)
    t = torch.from_numpy(a)
    if dtype == "bf16":
        t = t.to(torch.bfloat16)
    host = t.float().numpy()[:, :cols].astype(np.float64)
    dev = t.to(DEV)[:, :cols]
    return dev, host


def _same(got, want):
    """Equal as numbers (-0 == +0) and no NaN anywhere."""
    got = np.asarray(got, np.float64)
    assert not np.isnan(got).any()
    assert got.shape == want.shape
    np.testing.assert_array_equal(got, want)


CASES = [
    # name, rows, cols, dim, dtype, K, L (None: from recall 0.95), minimize, aggregate, pad, kind, override
    ("rows_ragged_topk", 37, 10007, 1, "fp32", 10, 176, False, True, 0, "normal", -1),
    ("rows_bins_of_32", 16, 65536, 1, "fp32", 10, 2048, False, False, 0, "normal", -1),
    ("rows_bins_under_4_min_ties", 8, 5000, 1, "fp32", 10, 1351, True, False, 0, "ints", -1),
    ("rows_L_eq_n", 5, 777, 1, "fp32", 20, 777, False, True, 0, "ints", -1),
    ("rows_one_bin", 6, 100003, 1, "fp32", 1, 1, False, True, 0, "normal", -1),
    ("rows_huge_bins_strided", 9, 50001, 1, "fp32", 3, 3, False, False, 13, "ints", -1),
    ("rows_items_of_many_bins", 3, 300000, 1, "fp32", 10, 20000, False, False, 0, "ints", -1),
    ("rows_bf16", 33, 20000, 1, "bf16", 10, 500, False, True, 0, "normal", -1),
    ("rows_bf16_unaligned_min", 7, 3001, 1, "bf16", 16, 300, True, True, 3, "ints", -1),
    ("rows_signed_zeros", 4, 4096, 1, "fp32", 8, 64, False, True, 0, "zeros", -1),
    ("rows_masked", 6, 9000, 1, "fp32", 10, 900, False, True, 0, "masked", -1),
    ("rows_recall_target", 12, 30000, 1, "fp32", 10, None, False, True, 0, "normal", -1),
    ("rows_override_shard", 12, 2816, 1, "fp32", 10, None, False, False, 0, "normal", 11264),
    ("cols_topk", 10003, 37, 0, "fp32", 10, 176, False, True, 0, "normal", -1),
    ("cols_bf16_min_bins", 4099, 300, 0, "bf16", 8, 64, True, False, 5, "ints", -1),
    ("cols_single_column", 5000, 1, 0, "fp32", 5, 5000, False, True, 0, "ints", -1),
    ("cols_masked", 3000, 70, 0, "fp32", 10, 40, False, True, 0, "masked", -1),
    ("cols_split_bins", 20000, 130, 0, "fp32", 10, 50, False, True, 0, "ints", -1),
    # top-K over more than 1024 bin winners: the key-range select, its byte-wise fallback
    # (thousands of equal winners in one bucket) and element strides (dimension 0)
    ("rows_select_range_min", 4, 200000, 1, "fp32", 100, 5000, True, True, 0, "normal", -1),
    ("rows_select_many_ties", 3, 300000, 1, "fp32", 10, 20000, False, True, 0, "ints", -1),
    ("cols_select_strided", 60000, 16, 0, "fp32", 50, 3000, False, True, 0, "normal", -1),
    ("cols_split_bf16_min_strided", 9001, 65, 0, "bf16", 5, 7, True, False, 3, "ints", -1),
    # top-K over 1025 .. 4096 winners with K <= 32 (ragged lengths, ties, minimisation,
    # strided columns)
    ("rows_block_select_ragged_ties_min", 7, 1100, 1, "fp32", 32, 1100, True, True, 0, "ints", -1),
    ("rows_block_select_16", 5, 3001, 1, "bf16", 17, 3001, False, True, 2, "normal", -1),
    ("rows_block_select_bins", 6, 40000, 1, "fp32", 10, 4096, False, True, 0, "ints", -1),
    ("cols_block_select_strided", 2500, 9, 0, "bf16", 10, 2500, False, True, 1, "ints", -1),
    # the largest K the op takes (1024): key-range select, one-wave select, columns
    ("rows_max_K_range_select", 5, 5000, 1, "fp32", 1024, 5000, False, True, 0, "normal", -1),
    ("rows_max_K_wave_select_ties", 3, 1024, 1, "fp32", 1024, 1024, True, True, 0, "ints", -1),
    ("cols_max_K_bf16", 2000, 7, 0, "bf16", 1024, 1500, False, True, 0, "normal", -1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_approx_top_k_matches_oracle(case):
    name, rows, cols, dim, dt, K, L, mn, agg, pad, kind, over = case
    _log(f"approx case {name}: rows={rows} cols={cols} dim={dim} {dt} K={K} L={L} min={mn} agg={agg}")
    dev, host = _inputs(rows, cols, kind, dt, pad, seed=100 + CASES.index(case))
    n = cols if dim == 1 else rows
    Lr = L if L is not None else oracle.approx_bins(n, K, 0.95, over)
    if L is None:
        assert knn.approx_bins(n, K, 0.95, over) == Lr
    v, i = knn.approx_top_k(dev, K, reduction_dimension=dim, aggregate_to_topk=agg, minimize=mn, L=L,
                            reduction_input_size_override=over)
    torch.cuda.synchronize()
    ov, oi = oracle.approx_top_k(host, K, Lr, dim=dim, minimize=mn, aggregate=agg)
    _same(v.cpu().numpy(), ov)
    np.testing.assert_array_equal(i.cpu().numpy(), oi)


def _planted_rows(rows, n, seed):
    """N(0, 1) rows whose entries in 16 runs of 64 spread evenly over the row are raised
    by 100 above all others: a sample taken at those runs would overstate the row's top
    (a case for any sampling shortcut in the select)."""
    a = datagen.score_matrix(rows, n, seed, "normal")
    for ch in range(16):
        s0 = (n - 64) * ch // 15
        a[:, s0:s0 + 64] += np.float32(100.0)
    return a


SELECT_CASES = [
    # name, rows, n (= L: one candidate per bin), K, minimize, kind
    ("long_normal_k512_min", 4, 8192, 512, True, "normal"),
    ("long_normal_k64_65536", 3, 65536, 64, False, "normal"),
    ("long_normal_k300", 5, 18750, 300, False, "normal"),
    ("long_ties_ints_fallback_cap", 3, 40000, 10, False, "ints"),
    ("long_ties_ints_k100", 4, 16384, 100, True, "ints"),
    ("long_planted_fallback_count", 3, 18750, 300, False, "planted"),
    ("long_above_max_n", 2, 65537, 50, False, "normal"),
    ("long_min_n", 3, 4096, 200, False, "masked"),
]


@pytest.mark.parametrize("case", SELECT_CASES, ids=[c[0] for c in SELECT_CASES])
def test_select_long_rows(case):
    """Top-K over 4096..65537 candidates per row (the key-range select): K up to 512,
    minimisation, thousands of exact ties, masked scores and a row whose evenly spread
    runs hold its largest values, bit for bit against the oracle."""
    name, rows, n, K, mn, kind = case
    _log(f"select case {name}: rows={rows} n={n} K={K} min={mn} {kind}")
    seed = 500 + SELECT_CASES.index(case)
    a = _planted_rows(rows, n, seed) if kind == "planted" else datagen.score_matrix(rows, n, seed, kind)
    dev = torch.from_numpy(a).to(DEV)
    v, i = knn.approx_top_k(dev, K, minimize=mn, L=n)
    torch.cuda.synchronize()
    ov, oi = oracle.approx_top_k(a.astype(np.float64), K, n, minimize=mn)
    _same(v.cpu().numpy(), ov)
    np.testing.assert_array_equal(i.cpu().numpy(), oi)


def test_approx_two_calls_and_min_wrapper():
    """Consecutive calls with different shapes on the same stream, and approx_min_k."""
    for rows, cols in ((64, 8192), (3, 1000)):
        dev, host = _inputs(rows, cols, "normal", "fp32", 0, seed=rows)
        v, i = knn.approx_min_k(dev, 5, L=100)
        ov, oi = oracle.approx_top_k(host, 5, 100, minimize=True)
        _same(v.cpu().numpy(), ov)
        np.testing.assert_array_equal(i.cpu().numpy(), oi)


@pytest.mark.parametrize("dt", ["fp32", "bf16"])
def test_approx_full_size_ablation_shape_sampled(dt):
    """The bins of a 1024 x 2^20 score matrix at L = 128 (the shape of the paper's
    reshape + argmax comparison), as the benchmark launches them; sampled rows are
    checked against the oracle."""
    w = datagen.ABLATION
    M, N, L = w["M"], w["N"], w["L"]
    _log(f"approx full-size {dt}: {M} x {N}, L={L}")
    S = datagen.normal_device(M, N, seed=77, dtype=torch.bfloat16 if dt == "bf16" else None)
    v, i = knn.approx_top_k(S, 10, L=L, aggregate_to_topk=False)
    vk, ik = knn.approx_top_k(S, 10, L=L)
    torch.cuda.synchronize()
    for r in (0, 1, 511, 1000, M - 1):
        host = S[r:r + 1].float().cpu().numpy().astype(np.float64)
        ov, oi = oracle.approx_top_k(host, 10, L, aggregate=False)
        _same(v[r:r + 1].cpu().numpy(), ov)
        np.testing.assert_array_equal(i[r:r + 1].cpu().numpy(), oi)
        ov, oi = oracle.approx_top_k(host, 10, L)
        _same(vk[r:r + 1].cpu().numpy(), ov)
        np.testing.assert_array_equal(ik[r:r + 1].cpu().numpy(), oi)
    del S, v, i, vk, ik
    torch.cuda.empty_cache()


def test_approx_full_size_dim0_sampled():
    """Reduction down the columns of a 2^20 x 1024 matrix at L = 128 (bins of 8192 rows,
    split over the waves of a workgroup), as the benchmark launches it; sampled columns
    against the oracle."""
    w = datagen.ABLATION
    M, N, L = w["M"], w["N"], w["L"]
    _log(f"approx full-size dim 0: {N} x {M}, L={L}")
    S = datagen.normal_device(N, M, seed=77)
    v, i = knn.approx_top_k(S, 10, reduction_dimension=0, L=L, aggregate_to_topk=False)
    torch.cuda.synchronize()
    for c in (0, 63, 64, 700, M - 1):
        host = S[:, c:c + 1].cpu().numpy().astype(np.float64)
        ov, oi = oracle.approx_top_k(host, 10, L, dim=0, aggregate=False)
        _same(v[:, c:c + 1].cpu().numpy(), ov)
        np.testing.assert_array_equal(i[:, c:c + 1].cpu().numpy(), oi)
    del S, v, i
    torch.cuda.empty_cache()
