"""GPU parity at the benchmark's full sizes, in the launch configurations the benchmark
times: sampled outputs are checked against the oracle (run on an MI355X).

  * cosine, GloVe-shaped (Q 10,000, N 1.2M, D 100, K 100, L 16,384): the FP32 search, and
    FP8 + FP32 rerank at two of the benchmark's (L, rerank depth) candidates;
  * the batched persistent launch over four BF16 databases (up to 16M x 256) with the
    autotuned plan, replayed from a captured graph: every batch equals a search of its
    database alone, and sampled queries of every database are checked against the oracle;
  * BF16 MIPS with K = 64, L = 32,768 over 4M x 256 rows, and the backward of the
    benchmark's loss: sampled dQ rows and dX rows against the oracle's FP64 gradient.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2206_14286_amd import datagen, knn
from parity import FP8_U, check_bins, check_rerank, check_topk

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dpad(D, compute):
    step = 64 if compute == "fp8" else 32
    return (D + step - 1) // step * step


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_full_size_cosine_glove_sampled():
    w = datagen.WORKLOADS["cosine_glove"]
    M, N, D, K, L = w["M"], w["N"], w["D"], w["K"], w["L"]
    _log(f"cosine_glove full size: generating {M} x {D} queries, {N} rows")
    Q, X = datagen.make("cosine_glove", seed=0)
    Qd, Xd = torch.from_numpy(Q).to(DEV), torch.from_numpy(X).to(DEV)
    sample = np.linspace(0, M - 1, 8).astype(np.int64)
    Qs = Q[sample]

    _log("cosine_glove fp32: search as timed, then with the bins")
    db = knn.Database(Xd, "cosine", "fp32")
    vals, idx = db.search(Qd, K, L)
    v2, i2, bv, bi = db.search(Qd, K, L, return_bins=True)
    torch.cuda.synchronize()
    assert torch.equal(idx, i2) and torch.equal(vals, v2)
    Qq = oracle.quantize_like_library(Qs, "cosine", "fp32")
    Xq = oracle.quantize_like_library(X, "cosine", "fp32")
    ora = oracle.search(Qq, Xq, "mips", L, K, bins=True)
    dp = _dpad(D, "fp32")
    n_sep, n_tie = check_bins(Qq, Xq, "mips", L, bv.cpu().numpy()[sample], bi.cpu().numpy()[sample], ora, dp)
    assert n_sep > 0.5 * (n_sep + n_tie)
    check_topk(Qq, Xq, "mips", K, vals.cpu().numpy()[sample], idx.cpu().numpy()[sample], ora, dp)
    del db, bv, bi, v2, i2
    _free()

    db8 = knn.Database(Xd, "cosine", "fp8")
    for Lc, Kr in ((L, 2 * K), (N // 64, 3 * K)):
        _log(f"cosine_glove fp8 + rerank: L={Lc} Kr={Kr}")
        vals, idx = db8.search(Qd, K, Lc, rerank=Kr)
        torch.cuda.synchronize()
        n_sure = check_rerank(Qs, X, "cosine", "fp8", K, Lc, Kr, vals.cpu().numpy()[sample],
                              idx.cpu().numpy()[sample], _dpad(D, "fp8"), FP8_U)
        _log(f"  {n_sure} sure rows checked")
        assert n_sure >= len(sample) * K // 4
    del db8, Xd, Qd, vals, idx
    _free()


def test_full_size_batched_autotuned_sampled():
    bf16 = torch.bfloat16
    _log("batched full size: generating", datagen.BATCHED_DBS)
    xs = [datagen.normal_device(n, d, seed=1000 + i, dtype=bf16) for i, (n, d) in enumerate(datagen.BATCHED_DBS)]
    dbs = [knn.Database(x, "mips", "bf16") for x in xs]
    sizes = datagen.batch_sizes(datagen.BATCHED_COUNT, seed=2)
    batches = []
    for b, m in enumerate(sizes):
        d = b % len(dbs)
        batches.append((datagen.normal_device(int(m), datagen.BATCHED_DBS[d][1], seed=2000 + b, dtype=bf16), d, 10))
    _log("batched: autotuning the plan")
    plan = knn.BatchedPlan(dbs, batches, recall_target=0.95, tune=True)
    info = plan.info()
    _log("plan", info)
    assert all(Ld >= oracle.bins_for_recall(10, 0.95) for Ld in info["L"])
    outs = plan.run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run()
    for ov, oi in outs:
        ov.zero_()
        oi.zero_()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    _log("batched: every batch against a search of its database alone")
    for b, ((Q, d, k), (ov, oi)) in enumerate(zip(batches, outs)):
        rv, ri = dbs[d].search(Q, k, int(info["L"][d]))
        torch.cuda.synchronize()
        assert torch.equal(oi, ri), f"batch {b}"
        assert torch.equal(ov, rv), f"batch {b}"
    for d, (n, D) in enumerate(datagen.BATCHED_DBS):
        b = next(b for b in range(d, len(batches), len(dbs)) if sizes[b] >= 2)
        Q = batches[b][0]
        qs = np.unique(np.array([0, Q.shape[0] - 1]))
        Ld = int(info["L"][d])
        _log(f"batched: database {d} ({n} x {D}, L={Ld}), batch {b}, queries {qs.tolist()} against the oracle")
        Xh = xs[d].cpu().float().numpy()
        Qs = Q.cpu().float().numpy()[qs]
        ora = oracle.search(Qs, Xh, "mips", Ld, 10, bins=True)
        ov, oi = outs[b]
        check_topk(Qs, Xh, "mips", 10, ov.cpu().numpy()[qs], oi.cpu().numpy()[qs], ora, _dpad(D, "bf16"))
        del Xh
    del graph, plan, dbs, xs, batches, outs, Q, ov, oi
    _free()


def test_full_size_mips_backward_sampled():
    w = datagen.WORKLOADS["mips_backward"]
    M, N, D, K, L = w["M"], w["N"], w["D"], w["K"], w["L"]
    bf16 = torch.bfloat16
    s = 1.0 / D ** 0.5
    _log(f"mips_backward full size: {M} queries, {N} x {D} rows, K={K}, L={L}")
    X = datagen.normal_device(N, D, seed=3000, scale=s, dtype=bf16)
    Q = datagen.normal_device(M, D, seed=3001, scale=s, dtype=bf16)
    db = knn.Database(X, "mips", "bf16")
    o = (torch.empty((M, K), dtype=torch.float32, device=DEV), torch.empty((M, K), dtype=torch.int32, device=DEV))
    db.search(Q, K, L, out=o)
    vals, idx = o
    v2, i2, bv, bi = db.search(Q, K, L, return_bins=True)
    torch.cuda.synchronize()
    assert torch.equal(idx, i2) and torch.equal(vals, v2)
    sample = np.linspace(0, M - 1, 8).astype(np.int64)
    _log("mips_backward: oracle on the sampled queries")
    Xh = X.cpu().float().numpy()  # BF16 values: the rows the kernel computes with
    Qh = Q.cpu().float().numpy()
    ora = oracle.search(Qh[sample], Xh, "mips", L, K, bins=True)
    dp = _dpad(D, "bf16")
    n_sep, n_tie = check_bins(Qh[sample], Xh, "mips", L, bv.cpu().numpy()[sample], bi.cpu().numpy()[sample], ora, dp)
    assert n_sep > 0.5 * (n_sep + n_tie)
    check_topk(Qh[sample], Xh, "mips", K, vals.cpu().numpy()[sample], idx.cpu().numpy()[sample], ora, dp)
    del bv, bi, v2, i2
    _free()

    _log("mips_backward: backward of the cross-entropy over the retrieved scores")
    t = torch.from_numpy(datagen.targets(M, K, seed=2)).to(DEV)
    g = torch.softmax(vals, dim=1)
    g[torch.arange(M, device=DEV), t] -= 1.0
    g = (g / M).contiguous()
    dQ = torch.empty((M, D), dtype=torch.float32, device=DEV)
    dX = torch.zeros((N, D), dtype=torch.float32, device=DEV)
    knn.backward(g, idx, Q, X, "mips", out=(dQ, dX))
    torch.cuda.synchronize()
    gh = g.cpu().numpy().astype(np.float64)
    ih = idx.cpu().numpy().astype(np.int64)
    # rows of dX to check: rows retrieved by the sampled queries, and rows nobody retrieved
    J = np.unique(ih[sample[:4], :8].ravel())
    unused = np.setdiff1d(np.arange(0, N, N // 64), ih.ravel())
    # every query that retrieved one of J contributes to it: solve the sub-problem of those
    # queries and the sampled ones over the rows they retrieved (indices relabelled)
    U = np.union1d(sample, np.nonzero(np.isin(ih, J).any(axis=1))[0])
    R = np.unique(ih[U].ravel())
    rq, rx = oracle.backward(gh[U], np.searchsorted(R, ih[U]), Qh[U], Xh[R], "mips")
    dQh = dQ.cpu().numpy()
    at = lambda a: 2e-5 * np.abs(a).max() * K ** 0.5
    np.testing.assert_allclose(dQh[sample], rq[np.searchsorted(U, sample)], rtol=0, atol=at(rq))
    dXJ = dX[torch.from_numpy(J).to(DEV)].cpu().numpy()
    np.testing.assert_allclose(dXJ, rx[np.searchsorted(R, J)], rtol=0, atol=at(rx))
    assert not dX[torch.from_numpy(unused).to(DEV)].any().item(), "a row nobody retrieved has a gradient"
    _log(f"  dQ rows {sample.size}, dX rows {J.size} (+{unused.size} untouched) checked; {U.size} queries in the sub-problem")
    del db, X, Q, dQ, dX, g, vals, idx, o
    _free()
