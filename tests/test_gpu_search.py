"""GPU parity of the HIP search path against the FP64 oracle (run on an MI355X)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2206_14286_amd import datagen, knn
from parity import FP8_U, check_bins, check_rerank, check_topk, gamma

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t.to(dtype) if dtype is not None else t


def make_inputs(metric, M, N, D, seed):
    if metric == "l2":
        return datagen.int_mixture(M, D, seed + 1, centres=16), datagen.int_mixture(N, D, seed, centres=16)
    return datagen.normal(M, D, seed + 1), datagen.normal(N, D, seed)


def dpad_of(D, compute):
    step = 64 if compute == "fp8" else 32
    return (D + step - 1) // step * step


# Unit roundoff used in the rounding bound per compute type.  FP32 and BF16 products
# are exact and the matrix unit accumulates in FP32: u = 2^-23 (twice the RNE unit).
# The FP8 instruction's bound is the measured one (parity.FP8_U).  Values are held to
# 1e-5 relative or the rounding bound, whichever is larger, for every compute type.
U_BOUND = {"fp32": 2.0 ** -23, "bf16": 2.0 ** -23, "fp8": FP8_U}
V_RTOL = {"fp32": 1e-5, "bf16": 1e-5, "fp8": 1e-5}


CASES = [
    # metric, M, N, D, K, L, compute
    ("mips", 64, 65536, 128, 10, 2048, "fp32"),   # the small MIPS workload in full
    ("mips", 70, 5003, 100, 7, 61, "fp32"),       # ragged N, L not dividing N, D padded
    ("l2", 300, 4099, 128, 10, 176, "fp32"),
    ("cosine", 129, 3001, 96, 5, 40, "fp32"),
    ("mips", 33, 777, 64, 3, 777, "fp32"),        # L = N: one row per bin
    ("mips", 5, 1000, 32, 4, 4, "fp32"),          # L = K: bins of 250 rows
    ("l2", 257, 2048, 256, 10, 64, "fp32"),
    ("mips", 1, 100, 16, 1, 1, "fp32"),           # one query, one bin
    ("mips", 200, 4096, 128, 10, 128, "bf16"),
    ("l2", 130, 3000, 128, 10, 100, "bf16"),
    ("cosine", 260, 2000, 256, 8, 73, "bf16"),
    ("cosine", 100, 3333, 100, 20, 300, "fp8"),
    ("mips", 64, 2500, 128, 10, 50, "fp8"),
    ("l2", 129, 1500, 64, 5, 1500, "fp8"),
    ("l2", 200, 3000, 64, 10, 80, "bf16"),         # bins of 37-38 rows: one boundary per tile
    ("mips", 100, 2000, 128, 5, 45, "fp8"),        # bins of 44-45 rows
    ("cosine", 64, 4100, 128, 10, 120, "fp32"),    # bins of 34-35 rows, ragged tail tile
    ("mips", 300, 3000, 192, 10, 50, "bf16"),      # depth 192: the single-accumulator form
    ("l2", 200, 2500, 256, 10, 40, "bf16"),        # depth 256, L2, bins of 62-63 rows
    # every remaining (compute type, depth, column blocks) kernel instance
    ("mips", 150, 2000, 192, 10, 70, "fp8"),       # FP8 depth 192: double-buffered form
    ("l2", 260, 3000, 256, 10, 90, "fp8"),         # FP8 depth 256: single-accumulator form
    ("cosine", 90, 2000, 250, 5, 64, "fp8"),       # FP8 depth 256, one column block
    ("mips", 140, 1800, 192, 8, 55, "fp32"),       # FP32 depth 192
    ("l2", 300, 2000, 20, 10, 100, "bf16"),        # BF16 depth 32
    ("mips", 100, 2222, 128, 10, 70, "bf16"),      # BF16 depth 128, one column block
    # at most 64 queries in FP32: the depth-split kernel (two wave pairs per query block)
    ("l2", 48, 3001, 256, 10, 100, "fp32"),        # depth 256, bins of 30-31 rows, ragged tail tile
    ("l2", 64, 2000, 96, 5, 37, "fp32"),           # depth 96, bins of 54-55 rows: one boundary per tile
    ("cosine", 20, 1500, 192, 6, 15, "fp32"),      # depth 192, one query wave, bins of 100 rows
    ("mips", 64, 4096, 64, 8, 16, "fp32"),         # depth 64, bins of 256 rows
    # fewer rows than one 32-row tile
    ("mips", 10, 5, 16, 2, 3, "fp32"),
    ("l2", 7, 31, 64, 5, 31, "bf16"),
    ("cosine", 5, 1, 8, 1, 1, "fp8"),
    ("mips", 40, 20, 100, 4, 7, "fp8"),
]


@pytest.mark.parametrize("metric,M,N,D,K,L,compute", CASES)
def test_bins_and_topk_vs_oracle(metric, M, N, D, K, L, compute):
    _log(f"case {metric} M={M} N={N} D={D} K={K} L={L} {compute}")
    Q, X = make_inputs(metric, M, N, D, seed=M + N)
    db = knn.Database(to_dev(X), metric, compute)
    vals, idx, bv, bi = db.search(to_dev(Q), K, L, return_bins=True)
    torch.cuda.synchronize()
    Qq = oracle.quantize_like_library(Q, metric, compute)
    Xq = oracle.quantize_like_library(X, metric, compute)
    mo = "mips" if metric == "cosine" else metric
    ora = oracle.search(Qq, Xq, mo, L, K, bins=True)
    dp = dpad_of(D, compute)
    u, rt = U_BOUND[compute], V_RTOL[compute]
    n_sep, n_tie = check_bins(Qq, Xq, mo, L, bv.cpu().numpy(), bi.cpu().numpy(), ora, dp, u=u, value_rtol=rt)
    assert n_sep > 0.5 * (n_sep + n_tie)
    check_topk(Qq, Xq, mo, K, vals.cpu().numpy(), idx.cpu().numpy(), ora, dp, u=u, value_rtol=rt)


LARGE_L_CASES = [
    # metric, M, N, D, K, L, compute, Kr: more than 1024 bins (the select's histogram
    # path), searched once with the bins kept internally and once with them returned
    ("mips", 70, 70000, 128, 10, 2050, "fp32", 0),     # L not a multiple of 16, ragged M
    ("l2", 300, 40000, 128, 10, 1500, "bf16", 0),      # bins of 26-27 rows
    ("cosine", 130, 65536, 128, 10, 2048, "fp8", 0),   # bins of 32 rows (small-bin FP8 kernel)
    ("mips", 257, 50000, 256, 8, 1100, "bf16", 0),     # depth 256
    ("l2", 129, 30000, 100, 5, 3000, "fp8", 64),       # with the FP32 rerank
    ("cosine", 40, 20000, 64, 10, 1025, "bf16", 100),  # one bin above the wave-select limit
    ("mips", 5, 20000, 64, 3, 1500, "fp32", 0),        # fewer rows than one group of 16
]


@pytest.mark.parametrize("metric,M,N,D,K,L,compute,Kr", LARGE_L_CASES)
def test_large_L_search(metric, M, N, D, K, L, compute, Kr):
    """A search that keeps its bins internally returns exactly what the same search
    returns when the caller takes the bins, and the top-K matches the oracle."""
    _log(f"large L {metric} M={M} N={N} D={D} K={K} L={L} {compute} Kr={Kr}")
    Q, X = make_inputs(metric, M, N, D, seed=M + N + L)
    db = knn.Database(to_dev(X), metric, compute)
    Qd = to_dev(Q)
    v1, i1 = db.search(Qd, K, L, rerank=Kr)
    v2, i2, bv, bi = db.search(Qd, K, L, rerank=Kr, return_bins=True)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2) and torch.equal(v1, v2)
    if Kr:
        return
    Qq = oracle.quantize_like_library(Q, metric, compute)
    Xq = oracle.quantize_like_library(X, metric, compute)
    mo = "mips" if metric == "cosine" else metric
    ora = oracle.search(Qq, Xq, mo, L, K, bins=True)
    u, rt = U_BOUND[compute], V_RTOL[compute]
    check_bins(Qq, Xq, mo, L, bv.cpu().numpy(), bi.cpu().numpy(), ora, dpad_of(D, compute), u=u, value_rtol=rt)
    check_topk(Qq, Xq, mo, K, v1.cpu().numpy(), i1.cpu().numpy(), ora, dpad_of(D, compute), u=u, value_rtol=rt)


@pytest.mark.parametrize("metric,compute", [(m, c) for m in ("mips", "l2", "cosine") for c in ("fp32", "bf16", "fp8")])
def test_prepared_rows_match_reference_quantisers(metric, compute):
    """The rows the kernel streams are bit-identical to the oracle's quantisers."""
    _log(f"prepare {metric} {compute}")
    N, D = 1000, 100
    X = datagen.normal(N, D, 5) * np.float32(3.0)
    X[7] = 0
    db = knn.Database(to_dev(X), metric, compute)
    codes, exps, hn = db.export()
    Xn = oracle.normalize_rows_f32(X) if metric == "cosine" else X
    if compute == "fp32":
        np.testing.assert_array_equal(codes.view(np.uint32), Xn.view(np.uint32))
        deq = Xn
    elif compute == "bf16":
        v, c = oracle.bf16_round(Xn)
        np.testing.assert_array_equal(codes, c)
        deq = v
    else:
        deq, c, e = oracle.fp8_quantize_rows(Xn)
        np.testing.assert_array_equal(exps, e)
        np.testing.assert_array_equal(codes, c)
    if metric == "l2":
        ref = 0.5 * (deq.astype(np.float64) ** 2).sum(1)
        np.testing.assert_allclose(hn, ref, rtol=2e-6, atol=1e-30)


def decode_query_tiles(buf, M, D, compute):
    """Rows of a prepared query buffer (the piece layout of the distance kernel's tiles):
    element codes (M x D) and the per-row FP8 scale exponents."""
    es = {"fp32": 4, "bf16": 2, "fp8": 1}[compute]
    dp = dpad_of(D, compute)
    ng = dp * es // 32
    tb = ng * 1024 + 256
    E = 16 // es
    raw = buf.cpu().numpy()
    cdt = {"fp32": np.uint32, "bf16": np.uint16, "fp8": np.uint8}[compute]
    codes = np.zeros((M, dp), cdt)
    exps = np.zeros(M, np.int64)
    for r in range(M):
        t, rr = divmod(r, 32)
        base = t * tb
        for g in range(ng):
            for hf in range(2):
                o = base + (rr // 4) * ng * 128 + g * 128 + hf * 64 + (rr % 4) * 16
                d0 = g * 2 * E + hf * E
                codes[r, d0:d0 + E] = raw[o:o + 16].view(cdt)
        exps[r] = int(raw[base + ng * 1024 + 128 + rr]) - 127
    return codes[:, :D], exps


@pytest.mark.parametrize("metric,compute", [(m, c) for m in ("mips", "l2", "cosine") for c in ("fp32", "bf16", "fp8")])
def test_prepared_queries_match_reference_quantisers(metric, compute):
    """The query rows the kernel reads are bit-identical to the oracle's quantisers."""
    _log(f"prepare queries {metric} {compute}")
    M, D = 77, 100
    Q = datagen.normal(M, D, 6) * np.float32(2.0)
    Q[5] = 0
    db = knn.Database(to_dev(datagen.normal(64, D, 7)), metric, compute)
    codes, exps = decode_query_tiles(db.prepare_queries(to_dev(Q)), M, D, compute)
    Qn = oracle.normalize_rows_f32(Q) if metric == "cosine" else Q
    if compute == "fp32":
        np.testing.assert_array_equal(codes, Qn.view(np.uint32))
    elif compute == "bf16":
        np.testing.assert_array_equal(codes, oracle.bf16_round(Qn)[1])
    else:
        _, c, e = oracle.fp8_quantize_rows(Qn)
        np.testing.assert_array_equal(exps, e)
        np.testing.assert_array_equal(codes, c)


def test_l2_integer_data_exact():
    """Integer data in [0, 255]: every FP32 (and BF16) partial sum is exact, so bins and
    top-K must equal the oracle's bit for bit, ties included (lowest row wins)."""
    M, N, D, K, L = 256, 20000, 128, 10, 176
    Q = datagen.int_mixture(M, D, 31)
    X = datagen.int_mixture(N, D, 30)
    ora = oracle.search(Q, X, "l2", L, K, bins=True)
    # 48 queries: the FP32 search takes the depth-split kernel (partial sums added in LDS)
    for compute, m in (("fp32", M), ("bf16", M), ("fp32", 48)):
        _log(f"l2 exact {compute} M={m}")
        db = knn.Database(to_dev(X), "l2", compute)
        vals, idx, bv, bi = db.search(to_dev(Q[:m]), K, L, return_bins=True)
        np.testing.assert_array_equal(bi.cpu().numpy(), ora["bin_i"][:m])
        np.testing.assert_array_equal(bv.cpu().numpy().astype(np.float64), ora["bin_v"][:m])
        np.testing.assert_array_equal(idx.cpu().numpy(), ora["top_i"][:m])
        np.testing.assert_array_equal(vals.cpu().numpy().astype(np.float64), ora["top_v"][:m])


@pytest.mark.parametrize("metric", ["mips", "l2", "cosine"])
def test_plain_search_entry_point_vs_oracle(metric):
    """knn_search (FP32 inputs, the database prepared inside the call) against the oracle."""
    M, N, D, K, L = 77, 5000, 96, 10, 250
    _log(f"plain knn_search {metric}")
    Q, X = make_inputs(metric, M, N, D, seed=91)
    v, i = knn.search(to_dev(Q), to_dev(X), K, L, metric)
    torch.cuda.synchronize()
    Qq = oracle.quantize_like_library(Q, metric, "fp32")
    Xq = oracle.quantize_like_library(X, metric, "fp32")
    mo = "mips" if metric == "cosine" else metric
    ora = oracle.search(Qq, Xq, mo, L, K, bins=True)
    check_topk(Qq, Xq, mo, K, v.cpu().numpy(), i.cpu().numpy(), ora, dpad_of(D, "fp32"), u=U_BOUND["fp32"],
               value_rtol=V_RTOL["fp32"])


def test_plain_search_entry_point():
    """knn_search (FP32 inputs, prepares X on every call) equals the prepared-database path."""
    Q = datagen.normal(100, 64, 41)
    X = datagen.normal(3000, 64, 40)
    for metric in ("mips", "l2", "cosine"):
        v1, i1 = knn.search(to_dev(Q), to_dev(X), 10, 100, metric)
        v2, i2 = knn.Database(to_dev(X), metric, "fp32").search(to_dev(Q), 10, 100)
        assert torch.equal(i1, i2) and torch.equal(v1, v2)


def test_zero_queries_is_noop():
    X = to_dev(datagen.normal(100, 16, 1))
    db = knn.Database(X, "mips")
    v, i = db.search(torch.empty((0, 16), device=DEV), 5, 10)
    assert v.shape == (0, 5)


@pytest.mark.parametrize("compute", ["bf16", "fp8"])
def test_rerank_recovers_recall(compute):
    """Low-precision GEMM + FP32 rerank of the best Kr bin winners: the returned scores are
    the FP32 scores of the original rows, and recall against the exact FP64 K-NN matches
    the FP64 approximate search at the same L."""
    metric = "cosine" if compute == "fp8" else "l2"
    M, N, D, K, L, Kr = 128, 30000, 128, 10, 400, 40
    if metric == "l2":
        Q, X = datagen.int_mixture(M, D, 51, centres=64), datagen.int_mixture(N, D, 50, centres=64)
    else:
        Q, X = datagen.unit_mixture(M, D, 51, centres=50), datagen.unit_mixture(N, D, 50, centres=50)
    _log(f"rerank {compute} {metric}")
    db = knn.Database(to_dev(X), metric, compute)
    vals, idx = db.search(to_dev(Q), K, L, rerank=Kr)
    vals, idx = vals.cpu().numpy(), idx.cpu().numpy()
    ora = oracle.search(Q, X, metric, L, K, exact=True)
    s64, mag = oracle.pair_scores(Q, X, metric, np.repeat(np.arange(M), K), idx.ravel())
    np.testing.assert_allclose(vals.ravel(), s64, rtol=1e-5, atol=1e-5 * float(np.max(np.abs(s64))))
    mn = oracle.minimize_for(metric)
    rec_gpu = oracle.recall_tie_aware(s64.reshape(M, K), ora["ex_v"], mn).mean()
    rec_ora = oracle.recall_tie_aware(ora["top_v"], ora["ex_v"], mn).mean()
    _log(f"recall gpu {rec_gpu:.4f} oracle-fp64 {rec_ora:.4f}")
    assert rec_gpu >= rec_ora - 0.01


def test_full_size_l2_sift_sample():
    """The L2 workload at full size (N = 1M, M = 10,000, L = 176) in FP32 and BF16; 24 sampled
    queries are checked against the oracle (integer data: exact)."""
    _log("l2_sift full size: generating")
    Q, X = datagen.make("l2_sift", seed=0)
    w = datagen.WORKLOADS["l2_sift"]
    K, L = w["K"], w["L"]
    Xd, Qd = to_dev(X), to_dev(Q)
    sample = np.linspace(0, Q.shape[0] - 1, 24).astype(np.int64)
    ora = oracle.search(Q[sample], X, "l2", L, K, bins=True)
    for compute in ("fp32", "bf16"):
        _log(f"l2_sift full size {compute}")
        db = knn.Database(Xd, "l2", compute)
        vals, idx, bv, bi = db.search(Qd, K, L, return_bins=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(bi.cpu().numpy()[sample], ora["bin_i"])
        np.testing.assert_array_equal(idx.cpu().numpy()[sample], ora["top_i"])
        np.testing.assert_array_equal(vals.cpu().numpy()[sample].astype(np.float64), ora["top_v"])
        del db


RERANK_CASES = [
    # metric, compute, input dtype, D, Kr
    ("l2", "bf16", "fp32", 128, 40),
    ("cosine", "fp8", "fp32", 100, 150),
    ("mips", "bf16", "bf16", 96, 64),
    ("mips", "fp8", "fp32", 256, 300),
    ("l2", "fp8", "bf16", 100, 600),
    ("mips", "bf16", "fp32", 33, 65),
    ("mips", "bf16", "fp32", 64, 1024),   # the largest rerank depth (= L)
]


@pytest.mark.parametrize("metric,compute,in_dtype,D,Kr", RERANK_CASES)
def test_rerank_matches_oracle(metric, compute, in_dtype, D, Kr):
    """Rerank parity against the oracle's definition (the top-Kr bin winners of the
    quantised search, rescored in FP64 from the original rows, best K kept), under the
    rounding bounds of both stages; the rules are listed in ``parity.check_rerank``."""
    M, N, K, L = 64, 20000, 10, 1024
    _log(f"rerank parity {metric} {compute} in={in_dtype} D={D} Kr={Kr}")
    if metric == "l2":
        Q, X = datagen.int_mixture(M, D, 71, centres=32), datagen.int_mixture(N, D, 70, centres=32)
    else:
        Q, X = datagen.normal(M, D, 71), datagen.normal(N, D, 70)
    if in_dtype == "bf16":  # the caller's rows are BF16: the "original" rows are their values
        X = oracle.bf16_round(X)[0].astype(np.float32)
        Q = oracle.bf16_round(Q)[0].astype(np.float32)
    tdt = torch.bfloat16 if in_dtype == "bf16" else torch.float32
    db = knn.Database(to_dev(X, tdt), metric, compute)
    vals, idx = db.search(to_dev(Q, tdt), K, L, rerank=Kr)
    n_sure_checked = check_rerank(Q, X, metric, compute, K, L, Kr, vals.cpu().numpy(), idx.cpu().numpy(),
                                  dpad_of(D, compute), U_BOUND[compute])
    _log(f"  {n_sure_checked} sure rows checked")
    assert n_sure_checked >= M * K // 4
