"""GPU tests of the batched persistent search (graph capture, autotuner) and the backward pass."""
import os
import sys
import tempfile

import numpy as np
import pytest
import torch

import oracle
from paper_2206_14286_amd import datagen, knn
from parity import check_topk

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(torch.bfloat16)


def _make_batched(seed=0):
    shapes = [(3000, 64), (5000, 96), (7000, 128), (2000, 256)]
    Xs = [bf16_dev(datagen.normal(n, d, seed + 10 * i)) for i, (n, d) in enumerate(shapes)]
    dbs = [knn.Database(x, "mips", "bf16") for x in Xs]
    sizes = [1, 3, 17, 64, 200, 1, 300, 5, 129, 33, 2, 90, 257, 7]
    ks = [10, 5, 10, 1, 10, 10, 7, 10, 10, 3, 10, 10, 10, 2]
    batches = []
    for b, m in enumerate(sizes):
        d = b % 4
        Q = bf16_dev(datagen.normal(m, shapes[d][1], seed + 100 + b))
        batches.append((Q, d, ks[b]))
    return dbs, batches


def _reference(dbs, batches, Ls):
    refs = []
    for Q, d, k in batches:
        v, i = dbs[d].search(Q, k, Ls[d])
        refs.append((v.clone(), i.clone()))
    return refs


def test_batched_equals_unbatched_and_replays_in_a_graph():
    dbs, batches = _make_batched()
    plan = knn.BatchedPlan(dbs, batches, recall_target=0.95, tune=False)
    info = plan.info()
    _log("plan", info)
    assert all(L >= oracle.bins_for_recall(10, 0.95) for L in info["L"])
    outs = plan.run()
    torch.cuda.synchronize()
    refs = _reference(dbs, batches, info["L"])
    for (ov, oi), (rv, ri) in zip(outs, refs):
        assert torch.equal(oi, ri)
        assert torch.equal(ov, rv)
    # the largest batch of each database against the oracle, under the parity rule
    # (BF16 rows: the oracle runs on the same values)
    for d in range(4):
        b = max((j for j in range(len(batches)) if batches[j][1] == d), key=lambda j: batches[j][0].shape[0])
        Q, _, k = batches[b]
        Qf = Q.float().cpu().numpy()
        Xf = dbs[d].X.float().cpu().numpy()
        ora = oracle.search(Qf, Xf, "mips", info["L"][d], k, bins=True)
        dp = (Xf.shape[1] + 31) // 32 * 32
        check_topk(Qf, Xf, "mips", k, outs[b][0].cpu().numpy(), outs[b][1].cpu().numpy(), ora, dp)
    # capture the whole batched search into one graph and replay it with eager work between
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run()
    for rep in range(3):
        for ov, oi in outs:
            ov.zero_()
            oi.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (ov, oi), (rv, ri) in zip(outs, refs):
            assert torch.equal(oi, ri), f"replay {rep}"
            assert torch.equal(ov, rv), f"replay {rep}"
        _ = torch.randn(1000, device=DEV).sum().item()  # unrelated eager work between replays


def test_batched_plan_with_a_large_group():
    """With own launches for groups of at least 2,048 work items, a plan where one
    database's batches qualify (5,000 queries x 176 one-bin chunks: 3,520 items) next to
    small groups that share the persistent launch: every batch equals its unbatched
    search, bit for bit, also on graph replays, and the large group's batches match the
    oracle."""
    shapes = [(60000, 128), (3000, 64), (4000, 96)]
    Xs = [bf16_dev(datagen.normal(n, d, 300 + i)) for i, (n, d) in enumerate(shapes)]
    dbs = [knn.Database(x, "mips", "bf16") for x in Xs]
    spec = [(0, 2000, 10), (1, 7, 10), (0, 3000, 10), (2, 130, 5), (1, 65, 3)]
    batches = [(bf16_dev(datagen.normal(m, shapes[d][1], 400 + b)), d, k) for b, (d, m, k) in enumerate(spec)]
    plan = knn.BatchedPlan(dbs, batches, recall_target=0.95, tune=False, own_launch_min_items=2048)
    info = plan.info()
    _log("plan", info)
    outs = plan.run()
    torch.cuda.synchronize()
    refs = _reference(dbs, batches, info["L"])
    for (ov, oi), (rv, ri) in zip(outs, refs):
        assert torch.equal(oi, ri)
        assert torch.equal(ov, rv)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run()
    for rep in range(2):
        for ov, oi in outs:
            ov.zero_()
            oi.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (ov, oi), (rv, ri) in zip(outs, refs):
            assert torch.equal(oi, ri), f"replay {rep}"
            assert torch.equal(ov, rv), f"replay {rep}"
    Xf = dbs[0].X.float().cpu().numpy()
    for b in (0, 2):
        Q, _, k = batches[b]
        sel = np.arange(0, Q.shape[0], 97)
        Qf = Q.float().cpu().numpy()[sel]
        ora = oracle.search(Qf, Xf, "mips", info["L"][0], k, bins=True)
        check_topk(Qf, Xf, "mips", k, outs[b][0].cpu().numpy()[sel], outs[b][1].cpu().numpy()[sel], ora, 128)


def test_autotuner_writes_cache_and_keeps_results_valid():
    dbs, batches = _make_batched(seed=7)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tune.json")
        plan = knn.BatchedPlan(dbs, batches, recall_target=0.95, tune=True, cache_path=path)
        assert os.path.exists(path) and os.path.getsize(path) > 10
        info = plan.info()
        _log("tuned", info)
        assert all(L >= oracle.bins_for_recall(10, 0.95) for L in info["L"])
        outs = plan.run()
        torch.cuda.synchronize()
        refs = _reference(dbs, batches, info["L"])
        for (ov, oi), (rv, ri) in zip(outs, refs):
            assert torch.equal(oi, ri)
        plan2 = knn.BatchedPlan(dbs, batches, recall_target=0.95, tune=True, cache_path=path)  # cache hit
        assert plan2.info() == info


@pytest.mark.parametrize("metric", ["mips", "l2", "cosine"])
@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_backward_vs_dense_reference(metric, dtype):
    M, N, D, K, L = 96, 5000, 100, 16, 400
    Q = datagen.normal(M, D, 61)
    X = datagen.normal(N, D, 60)
    tq = torch.from_numpy(Q).to(DEV)
    tx = torch.from_numpy(X).to(DEV)
    if dtype == "bf16":
        tq, tx = tq.to(torch.bfloat16), tx.to(torch.bfloat16)
        Q, X = tq.float().cpu().numpy(), tx.float().cpu().numpy()
    db = knn.Database(tx, metric, dtype)
    _, idx = db.search(tq, K, L)
    g = torch.from_numpy(datagen.normal(M, K, 62)).to(DEV)
    dQ, dX = knn.backward(g, idx, tq, tx, metric)
    rq, rx = oracle.backward(g.cpu().numpy(), idx.cpu().numpy(), Q, X, metric)
    sq = np.abs(rq).max()
    sx = np.abs(rx).max()
    np.testing.assert_allclose(dQ.cpu().numpy(), rq, rtol=0, atol=2e-5 * sq * K ** 0.5)
    np.testing.assert_allclose(dX.cpu().numpy(), rx, rtol=0, atol=2e-5 * sx * K ** 0.5)


def test_autograd_cross_entropy_matches_fd_reference():
    """Softmax cross-entropy over the retrieved scores with a random retrieved target
    (Q = 8, N = 4096, D = 16, K = 64, L = 1024): autograd through the HIP backward equals
    the oracle's dense gradient, which is itself pinned to finite differences."""
    M, N, D, K, L = 8, 4096, 16, 64, 1024
    Q = datagen.normal(M, D, 101)
    X = datagen.normal(N, D, 100)
    t = torch.from_numpy(datagen.targets(M, K, 102)).to(DEV)
    tq = torch.from_numpy(Q).to(DEV).requires_grad_(True)
    tx = torch.from_numpy(X).to(DEV).requires_grad_(True)
    vals, idx = knn.knn(tq, tx, K, L, "mips")
    loss = torch.nn.functional.cross_entropy(vals, t)
    loss.backward()
    s = vals.detach().double().cpu().numpy()
    p = np.exp(s - s.max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    gg = p.copy()
    gg[np.arange(M), t.cpu().numpy()] -= 1.0
    gg /= M
    rq, rx = oracle.backward(gg, idx.cpu().numpy(), Q, X, "mips")
    np.testing.assert_allclose(tq.grad.cpu().numpy(), rq, rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(tx.grad.cpu().numpy(), rx, rtol=1e-4, atol=1e-6)
