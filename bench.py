#!/usr/bin/env python3
"""Throughput of the approximate K-NN search on one MI355X.

Workload (default): relaxed-L2 search, M = 10,000 queries against N = 1,000,000 rows,
D = 128, K = 10, L = 176 bins (the smallest L with ((L-1)/L)^(K-1) >= 0.95), on
SIFT1M-shaped synthetic data (integers in [0, 255] from a 256-centre Gaussian mixture).

One step = one pass of the hot path over the whole query batch, inputs resident in
HBM: query preparation + distance GEMM with the bin-reduce epilogue + top-K select
(+ FP32 rerank of the best K_r bin winners for the BF16 / FP8 forms; for the headline
form K_r is the smallest of K, 2K, 4K that keeps the method's own recall at L on the
recall sample, unless `--rerank` fixes it).  The
database is prepared once outside the timed region, as the paper precomputes the L2
half norms.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "queries/s at recall@10≥0.95 (N=1M,D=128) + % MFMA peak; BF16/FP8 vs FP32"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}  # MI355X dense matrix peaks
HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that determine the distance kernel's machine code and launch shape: the
# hardware counter figures under profiles/ are only reported while these are unchanged.
KERNEL_SOURCES = ["paper_2206_14286_amd/csrc/knn_fused.hip", "paper_2206_14286_amd/csrc/knn_internal.h",
                  "paper_2206_14286_amd/csrc/knn_common.cuh", "paper_2206_14286_amd/csrc/knn_api.cpp",
                  "paper_2206_14286_amd/build.py"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "fused_l2_sift_counters.md")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_figure(key):
    """A machine-readable figure of the committed rocprofv3 counter summary of the distance
    kernel on l2_sift, if the summary was taken on the current sources."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    vals = {}
    for line in open(COUNTERS_FILE):
        line = line.strip()
        if line.startswith("- source_sha256:"):
            vals["sha"] = line.split(":", 1)[1].strip()
        elif line.startswith(f"- {key}:"):
            vals["v"] = float(line.split(":", 1)[1].strip())
    if vals.get("sha") != kernel_source_digest() or "v" not in vals:
        return None
    return vals["v"]


def measured_traffic(compute):
    """HBM bytes per launch of the distance kernel for `compute` (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy of known size)."""
    return _counter_figure(f"traffic_bytes_per_launch[{compute}]")


def measured_cops(compute):
    """VALU lane-operations per score of the distance kernel (SQ_INSTS_VALU minus
    SQ_INSTS_MFMA, times 64 lanes, over M x N scores): the kernel's measured C."""
    return _counter_figure(f"valu_ops_per_score[{compute}]")


def perf_model_rows(line):
    """The performance model of Sec. 4 (eq. roofline) for every measured launch of the
    distance kernel in this run, in the layout of Table 2."""
    from paper_2206_14286_amd import perf_model as pm
    rows = []
    c = line["config"]

    def ib(M):
        return 256 if M > 128 else 128

    forms = {line["dtype"]: {"fused_tflops": line["roofline"]["achieved"], "L": c["L"]}}
    forms.update(line.get("variants", {}))
    for comp, r in forms.items():
        same_L = r["L"] == c["L"]
        rows.append(pm.entry("l2_sift", comp, "l2", c["M"], c["N"], dpad(c["D"], comp), r["L"], ib(c["M"]),
                             r["fused_tflops"], measured_traffic(comp) if same_L else None,
                             measured_cops(comp) if same_L else None,
                             _counter_figure(f"est_clock_ghz[{comp}]") if same_L else None))
    if "fp8_equal_recall" in line:
        r = line["fp8_equal_recall"]
        rows.append(pm.entry("l2_sift (FP8 at the FP32 recall)", "fp8", "l2", c["M"], c["N"], dpad(c["D"], "fp8"),
                             r["L"], ib(c["M"]), r["fused_tflops"]))
    o = line.get("other_workloads", {})
    if "mips_small" in o:
        r = o["mips_small"]
        rows.append(pm.entry("mips_small (whole call)", "fp32", "mips", r["M"], r["N"], r["D"], r["L"], ib(r["M"]),
                             r["tflops"]))
    if "cosine_glove" in o:
        r = o["cosine_glove"]
        for comp in ("fp32", "fp8"):
            if comp in r:
                rows.append(pm.entry("cosine_glove", comp, "cosine", r["M"], r["N"], dpad(r["D"], comp), r[comp]["L"],
                                     ib(r["M"]), r[comp]["tflops"]))
    if "batched" in o and "per_database" in o["batched"]:
        for r in o["batched"]["per_database"]:
            rows.append(pm.entry(f"batched database {r['N']} x {r['D']} ({r['queries']} queries)", "bf16", "mips",
                                 r["queries"], r["N"], dpad(r["D"], "bf16"), r["L"], r["qblock"], r["tflops"]))
    if "mips_backward" in o:
        r = o["mips_backward"]
        rows.append(pm.entry("mips_backward (forward)", "bf16", "mips", r["M"], r["N"], r["D"], r["L"], ib(r["M"]),
                             r["forward_tflops"]))
        if "backward_ms" in r:
            # dQ and dX: 2 M K D FLOP each; bytes: the gathered rows (X rows for dQ, Q rows for
            # dX, BF16), g and the indices, dQ written, dX read and written by the atomics
            M, K, D = r["M"], r["K"], r["D"]
            flops = 4.0 * M * K * D
            nbytes = 2.0 * M * K * D * 2 + M * K * 8 + M * D * 4 + 2.0 * M * K * D * 4
            rows.append(pm.entry_memory("mips_backward (backward kernels)", flops, nbytes, r["backward_ms"] * 1e-3))
    if "ablation" in o:
        r = o["ablation"]
        for comp in ("fp32", "bf16"):
            rows.append(pm.entry("ablation (fused)", comp, "mips", r["M"], r["N"], r["D"], r["L"], ib(r["M"]),
                                 r[comp]["fused_tflops"]))
    return rows


def dpad(D, compute):
    step = 64 if compute == "fp8" else 32
    return (D + step - 1) // step * step


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_kernel_events(fn, reps):
    """Average duration of fn's launches measured with HIP events on torch's current
    stream (the stream the library launches on)."""
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps / 1e3


def run_variant(knn, Xd, Qd, w, compute, rerank, steps, warmup, sample_idx, L=None):
    import torch
    M, N, D, K = Qd.shape[0], Xd.shape[0], w["D"], w["K"]
    L = w["L"] if L is None else L
    t0 = time.perf_counter()
    db = knn.Database(Xd, w["metric"], compute)
    prep_s = time.perf_counter() - t0
    out = (torch.empty((M, K), dtype=torch.float32, device="cuda"), torch.empty((M, K), dtype=torch.int32, device="cuda"))

    ws = torch.empty(db.workspace_size(M, K, L, rerank), dtype=torch.uint8, device="cuda")

    def step():
        db.search(Qd, K, L, rerank=rerank, out=out, workspace=ws)

    sec = time_steps(step, steps, warmup)
    # the distance + bin-reduce kernel alone, on prepared queries
    qbuf = db.prepare_queries(Qd)
    bins = (torch.empty((M, L), dtype=torch.float32, device="cuda"), torch.empty((M, L), dtype=torch.int32, device="cuda"))
    ksec = time_kernel_events(lambda: db.partial_reduce(qbuf, M, L, out=bins, resolve=False), max(steps, 5))
    flops = 2.0 * M * N * dpad(D, compute)
    res = {
        "compute": compute,
        "L": L,
        "rerank_k": rerank,
        "ms_per_step": sec * 1e3,
        "queries_per_s": M / sec,
        "fused_kernel_ms": ksec * 1e3,
        "fused_tflops": flops / ksec / 1e12,
        "fused_frac_of_peak": flops / ksec / 1e12 / PEAK_TFLOPS[compute],
        "db_prepare_ms": prep_s * 1e3,
        "idx_sample": out[1][sample_idx].cpu().numpy(),
        "val_sample": out[0][sample_idx].cpu().numpy(),
    }
    del db, qbuf, bins, ws
    torch.cuda.empty_cache()
    return res


# --------------------------------------------------------------------------- other workloads
def kernel_frac(flops, sec, compute):
    return {"tflops": flops / sec / 1e12, "frac_of_peak": flops / sec / 1e12 / PEAK_TFLOPS[compute]}


def row_mips_small(torch, knn, datagen, reps=200):
    """Plain FP32 entry point (knn_search) on the small MIPS workload: microseconds per call
    (database preparation included, as the plain entry point takes raw FP32 rows)."""
    w = datagen.WORKLOADS["mips_small"]
    Q, X = datagen.make("mips_small", seed=0)
    Qd, Xd = torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda()
    K, L = w["K"], w["L"]
    sec = time_kernel_events(lambda: knn.search(Qd, Xd, K, L, "mips"), reps)
    M, N = Q.shape[0], X.shape[0]
    # the same search against the database prepared once (knn_db_prepare + knn_db_search)
    db = knn.Database(Xd, "mips", "fp32")
    ws = torch.empty(db.workspace_size(M, K, L), dtype=torch.uint8, device="cuda")
    o = (torch.empty((M, K), dtype=torch.float32, device="cuda"), torch.empty((M, K), dtype=torch.int32, device="cuda"))
    psec = time_kernel_events(lambda: db.search(Qd, K, L, out=o, workspace=ws), reps)
    return {"workload": "mips_small", "M": M, "N": N, "D": w["D"], "K": K, "L": L, "compute": "fp32",
            "us_per_call": sec * 1e6, "queries_per_s": M / sec, **kernel_frac(2.0 * M * N * 128, sec, "fp32"),
            "prepared_us_per_call": psec * 1e6, "prepared_queries_per_s": M / psec}


def row_cosine_glove(torch, knn, datagen, oracle, steps, warmup, sample_n=256):
    """GloVe-shaped cosine search (K = 100, L = 16,384): FP32 plain against FP8 + FP32 rerank.
    The FP8 form takes the first (L, rerank depth) of a short list, in increasing cost,
    that reaches the FP32 form's recall on the sample (a deeper rerank, more bins)."""
    w = datagen.WORKLOADS["cosine_glove"]
    Q, X = datagen.make("cosine_glove", seed=0)
    Qd, Xd = torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda()
    M, N, D, K, L = Q.shape[0], X.shape[0], w["D"], w["K"], w["L"]
    sample = np.sort(np.random.default_rng(3).choice(M, sample_n, replace=False))
    st = torch.from_numpy(sample).cuda()
    log("cosine_glove: oracle exact on", sample_n, "queries")
    ex = oracle.search(Q[sample], X, "cosine", L, K, exact=True)
    exv = ex["ex_v"]

    def recall_of(idx):
        s64, _ = oracle.pair_scores(Q[sample], X, "cosine", np.repeat(np.arange(sample_n), K), idx.ravel())
        return float(oracle.recall_tie_aware(s64.reshape(-1, K), exv, False).mean())

    out = {"workload": "cosine_glove", "M": M, "N": N, "D": D, "K": K, "L": L,
           "oracle_fp64_recall_tie_aware": float(oracle.recall_tie_aware(ex["top_v"], exv, False).mean())}
    o = (torch.empty((M, K), dtype=torch.float32, device="cuda"), torch.empty((M, K), dtype=torch.int32, device="cuda"))
    bins = (torch.empty((M, L), dtype=torch.float32, device="cuda"), torch.empty((M, L), dtype=torch.int32, device="cuda"))
    for compute in ("fp32", "fp8"):
        db = knn.Database(Xd, "cosine", compute)
        rr, Lc = 0, L
        if compute == "fp8":
            # more bins as bins of 2^W rows (Algorithm 1's ShiftRight form) where N allows:
            # 64- and 32-row bins keep every bin boundary on a 32-row tile edge
            more = [N // r if N % r == 0 else m * L for r, m in ((64, 2), (32, 4))]
            for Lc, rr in ((L, 2 * K), (L, 4 * K), (more[0], 2 * K), (more[0], 3 * K), (more[0], 4 * K),
                           (more[1], 2 * K), (more[1], 4 * K)):
                rec = recall_of(db.search(Qd[st], K, Lc, rerank=rr)[1].cpu().numpy())
                log(f"  fp8 L={Lc} rerank {rr}: recall {rec:.4f}")
                if rec >= out["fp32"]["recall_tie_aware"]:
                    break
        if Lc != L:
            bins = (torch.empty((M, Lc), dtype=torch.float32, device="cuda"),
                    torch.empty((M, Lc), dtype=torch.int32, device="cuda"))
        ws = torch.empty(db.workspace_size(M, K, Lc, rr), dtype=torch.uint8, device="cuda")
        sec = time_steps(lambda: db.search(Qd, K, Lc, rerank=rr, out=o, workspace=ws), steps, warmup)
        rec = recall_of(o[1][st].cpu().numpy())
        qbuf = db.prepare_queries(Qd)
        ksec = time_kernel_events(lambda: db.partial_reduce(qbuf, M, Lc, out=bins, resolve=False), max(steps, 3))
        out[compute] = {"L": Lc, "rerank_k": rr, "ms_per_step": sec * 1e3, "queries_per_s": M / sec,
                        "recall_tie_aware": rec, "fused_kernel_ms": ksec * 1e3,
                        **kernel_frac(2.0 * M * N * dpad(D, compute), ksec, compute)}
        log(f"  cosine_glove {compute}: {out[compute]}")
        del db, qbuf, ws
        torch.cuda.empty_cache()
    return out


def row_batched(torch, knn, datagen, steps):
    """256 query batches (log-uniform sizes in [1, 4096]) against four BF16 databases in one
    persistent launch, replayed from a captured graph; the plan from the fixed heuristic and
    the plan the autotuner picks (it times candidate L and chunk sizes per database).  Beside
    them (not the row's figure): the heuristic plan with own launches for database groups of
    at least 2,048 work items (knn_plan_set_own_launches).
    Roofline: per database the larger of its MFMA time and one read of its rows, summed."""
    bf16 = torch.bfloat16
    xs = [datagen.normal_device(n, d, seed=1000 + i, dtype=bf16) for i, (n, d) in enumerate(datagen.BATCHED_DBS)]
    dbs = [knn.Database(x, "mips", "bf16") for x in xs]
    sizes = datagen.batch_sizes(datagen.BATCHED_COUNT, seed=2)
    batches = []
    for b, m in enumerate(sizes):
        d = b % len(dbs)
        batches.append((datagen.normal_device(int(m), datagen.BATCHED_DBS[d][1], seed=2000 + b, dtype=bf16), d, 10))
    bound = 0.0
    flops = 0.0
    for d, (n, dd) in enumerate(datagen.BATCHED_DBS):
        f = sum(2.0 * int(m) * n * dpad(dd, "bf16") for b, m in enumerate(sizes) if b % len(dbs) == d)
        flops += f
        bound += max(f / (PEAK_TFLOPS["bf16"] * 1e12), n * dpad(dd, "bf16") * 2 / (HBM_GBS * 1e9))
    nq = int(sizes.sum())
    out = {"workload": "batched", "batches": len(sizes), "queries": nq, "databases": datagen.BATCHED_DBS,
           "roofline_bound_ms": bound * 1e3}
    for name, tune, own in (("heuristic", False, 0), ("autotuned", True, 0), ("own_launches", False, 2048)):
        t0 = time.perf_counter()
        plan = knn.BatchedPlan(dbs, batches, recall_target=0.95, tune=tune, own_launch_min_items=own)
        create_s = time.perf_counter() - t0
        plan.run()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run()
        sec = time_steps(graph.replay, steps, 1)
        out[name] = {"plan": plan.info(), "plan_create_s": create_s, "ms_per_run": sec * 1e3,
                     "queries_per_s": nq / sec, "tflops": flops / sec / 1e12, "frac_of_roofline": bound / sec}
        del graph, plan
    best = min(("heuristic", "autotuned"), key=lambda k: out[k]["ms_per_run"])
    out.update({k: out[best][k] for k in ("ms_per_run", "queries_per_s", "tflops", "frac_of_roofline")})
    out["plan_used"] = best
    # each database's batches alone (one persistent launch each, the heuristic plan), for
    # the per-database rows of the performance model
    per_db = []
    for d, (n, dd) in enumerate(datagen.BATCHED_DBS):
        sub = [bt for bt in batches if bt[1] == d]
        plan = knn.BatchedPlan([dbs[d]], [(q, 0, k) for q, _, k in sub], recall_target=0.95, tune=False)
        plan.run()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run()
        sec = time_steps(graph.replay, steps, 1)
        m = sum(int(q.shape[0]) for q, _, _ in sub)
        f = 2.0 * m * n * dpad(dd, "bf16")
        info = plan.info()
        per_db.append({"N": n, "D": dd, "queries": m, "L": info["L"][0], "qblock": info["qblock"][0],
                       "ms_per_run": sec * 1e3, "tflops": f / sec / 1e12,
                       "frac_of_roofline": max(f / (PEAK_TFLOPS["bf16"] * 1e12), n * dpad(dd, "bf16") * 2 /
                                               (HBM_GBS * 1e9)) / sec})
        del graph, plan
    out["per_database"] = per_db
    del dbs, xs, batches
    torch.cuda.empty_cache()
    return out


def row_mips_backward(torch, knn, datagen, steps):
    """Forward BF16 search (K = 64, L = 32,768) and the backward of a softmax cross-entropy over
    the retrieved scores (random target per query), through the autograd Function
    (knn.KNN.apply: the search, then dQ gather and dX scatter-add in its backward); also the
    forward search and the backward kernels alone."""
    w = datagen.WORKLOADS["mips_backward"]
    M, N, D, K, L = w["M"], w["N"], w["D"], w["K"], w["L"]
    bf16 = torch.bfloat16
    s = 1.0 / D ** 0.5
    X = datagen.normal_device(N, D, seed=3000, scale=s, dtype=bf16)
    Q = datagen.normal_device(M, D, seed=3001, scale=s, dtype=bf16)
    db = knn.Database(X, "mips", "bf16")
    t = torch.from_numpy(datagen.targets(M, K, seed=2)).cuda()
    Qp = Q.clone().requires_grad_(True)
    Xp = X.requires_grad_(True)

    def autograd_step():
        Qp.grad = None
        Xp.grad = None
        vals, _ = knn.KNN.apply(Qp, Xp, K, L, "mips", db)
        torch.nn.functional.cross_entropy(vals, t).backward()

    asec = time_steps(autograd_step, steps, 1)
    o = (torch.empty((M, K), dtype=torch.float32, device="cuda"), torch.empty((M, K), dtype=torch.int32, device="cuda"))
    ws = torch.empty(db.workspace_size(M, K, L), dtype=torch.uint8, device="cuda")
    fsec = time_steps(lambda: db.search(Q, K, L, out=o, workspace=ws), steps, 1)
    vals, idx = o
    g = torch.softmax(vals, dim=1)
    g[torch.arange(M, device="cuda"), t] -= 1.0
    g = (g / M).contiguous()
    dQ = torch.empty((M, D), dtype=torch.float32, device="cuda")
    dX = torch.zeros((N, D), dtype=torch.float32, device="cuda")
    bsec = time_steps(lambda: knn.backward(g, idx, Q, X.detach(), "mips", out=(dQ, dX)), steps, 1)
    gathered = M * K * D * 2.0 * 2  # X rows for dQ and Q rows for dX, BF16
    atomics = M * K * D
    res = {"workload": "mips_backward", "M": M, "N": N, "D": D, "K": K, "L": L,
           "autograd_step_ms": asec * 1e3,
           "autograd_step_note": "KNN.apply forward + cross-entropy + backward (dQ, dX zeroed and "
                                 "accumulated in FP32, cast to the inputs' BF16), one step",
           "forward_ms": fsec * 1e3, "forward_queries_per_s": M / fsec,
           **{"forward_" + k: v for k, v in kernel_frac(2.0 * M * N * D, fsec, "bf16").items()},
           "backward_ms": bsec * 1e3, "backward_atomics_per_s": atomics / bsec,
           "backward_gb_s": (gathered + atomics * 4.0) / bsec / 1e9,
           "backward_frac_of_hbm": (gathered + atomics * 4.0) / bsec / 1e9 / HBM_GBS}
    del db, X, Q, Qp, Xp, dX, dQ, ws
    torch.cuda.empty_cache()
    return res


def row_approx(torch, knn, datagen, reps=10):
    """The approx_max_k op on a score matrix the caller holds (1024 x 2^20, the shape of
    the paper's reshape + argmax comparison), bins only (L = 128) and with the top-10:
    bound by HBM bandwidth, one read of the matrix per call."""
    w = datagen.ABLATION
    M, N, L = w["M"], w["N"], w["L"]
    out = {"workload": "approx_max_k", "rows": M, "cols": N, "L": L}
    for dt in ("fp32", "bf16"):
        S = datagen.normal_device(M, N, seed=77, dtype=torch.bfloat16 if dt == "bf16" else None)
        nbytes = S.numel() * S.element_size()
        ob = (torch.empty((M, L), dtype=torch.float32, device="cuda"), torch.empty((M, L), dtype=torch.int32, device="cuda"))
        ok = (torch.empty((M, 10), dtype=torch.float32, device="cuda"), torch.empty((M, 10), dtype=torch.int32, device="cuda"))
        tb = time_kernel_events(lambda: knn.approx_top_k(S, 10, L=L, aggregate_to_topk=False, out=ob), reps)
        tk = time_kernel_events(lambda: knn.approx_top_k(S, 10, L=L, out=ok), reps)
        out[dt] = {"bins_ms": tb * 1e3, "bins_gb_s": nbytes / tb / 1e9, "bins_frac_of_hbm": nbytes / tb / 1e9 / HBM_GBS,
                   "topk_ms": tk * 1e3, "topk_gb_s": nbytes / tk / 1e9}
        del S
        torch.cuda.empty_cache()
    # the same reduction down the columns of the transposed matrix (reduction_dimension 0)
    S = datagen.normal_device(N, M, seed=77)
    nbytes = S.numel() * S.element_size()
    ob = (torch.empty((L, M), dtype=torch.float32, device="cuda"), torch.empty((L, M), dtype=torch.int32, device="cuda"))
    tb = time_kernel_events(lambda: knn.approx_top_k(S, 10, reduction_dimension=0, L=L, aggregate_to_topk=False,
                                                     out=ob), reps)
    out["fp32_dim0"] = {"bins_ms": tb * 1e3, "bins_gb_s": nbytes / tb / 1e9,
                        "bins_frac_of_hbm": nbytes / tb / 1e9 / HBM_GBS}
    del S
    torch.cuda.empty_cache()
    return out


def row_ablation(torch, knn, datagen, reps=5):
    """The paper's comparison of the fused op with a dense GEMM + reshape + argmax (queries
    1024 x 128, database 2^20 x 128, L = 128, MIPS, FP32; also BF16): the fused distance +
    bin-reduce kernel against (a) a torch matmul (hipBLASLt) materialising the 1024 x 2^20
    scores, then this library's bin reduce on them, and (b) the same matmul, then torch's
    own reshape + max per bin, as the paper's listing does."""
    w = datagen.ABLATION
    M, N, D, L = w["M"], w["N"], w["D"], w["L"]
    Q = datagen.normal_device(M, D, seed=78)
    X = datagen.normal_device(N, D, seed=79)
    out = {"workload": "ablation", "M": M, "N": N, "D": D, "L": L}
    for dt in ("fp32", "bf16"):
        tdt = torch.float32 if dt == "fp32" else torch.bfloat16
        Qc, Xc = Q.to(tdt), X.to(tdt)
        db = knn.Database(Xc, "mips", dt)
        qbuf = db.prepare_queries(Qc)
        bins = (torch.empty((M, L), dtype=torch.float32, device="cuda"), torch.empty((M, L), dtype=torch.int32, device="cuda"))
        t_fused = time_kernel_events(lambda: db.partial_reduce(qbuf, M, L, out=bins, resolve=True), reps)
        S = torch.empty((M, N), dtype=tdt, device="cuda")
        XT = Xc.t().contiguous()
        t_gemm = time_kernel_events(lambda: torch.matmul(Qc, XT, out=S), reps)
        t_ours = time_kernel_events(lambda: knn.approx_top_k(S, 1, L=L, aggregate_to_topk=False, out=bins), reps)
        t_torch = time_kernel_events(lambda: torch.max(S.view(M, L, N // L), dim=2), reps)
        flops = 2.0 * M * N * D
        out[dt] = {"fused_ms": t_fused * 1e3, "fused_tflops": flops / t_fused / 1e12,
                   "gemm_ms": t_gemm * 1e3, "gemm_tflops": flops / t_gemm / 1e12,
                   "unfused_ours_ms": (t_gemm + t_ours) * 1e3, "unfused_reshape_argmax_ms": (t_gemm + t_torch) * 1e3,
                   "speedup_vs_unfused_ours": (t_gemm + t_ours) / t_fused,
                   "speedup_vs_reshape_argmax": (t_gemm + t_torch) / t_fused}
        del db, qbuf, S, XT, Qc, Xc
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--compute", default="bf16", choices=["fp32", "bf16", "fp8"], help="headline compute type")
    ap.add_argument("--rerank", default="auto",
                    help="bin winners rescored in FP32 for the headline low-precision form; 'auto': the "
                         "smallest of K, 2K, 4K whose recall on the sample reaches the FP64 oracle's at L")
    ap.add_argument("--variants", default="fp32,fp8", help="other compute types to time next to the headline")
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rows", default="fp8_equal_recall,exact_expectation_L,mips_small,cosine_glove,batched,"
                                      "mips_backward,approx,ablation",
                    help="other measurements to add to the line (empty: none)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a known-size kernel for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (sharding is a design only); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_2206_14286_amd import datagen, knn

    knn.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    name = "l2_sift"
    w = dict(datagen.WORKLOADS[name])
    log("generating", name)
    Q, X = datagen.make(name, seed=0)
    M, N, D, K, L = Q.shape[0], X.shape[0], w["D"], w["K"], w["L"]
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(M, args.recall_sample, replace=False))
    sample_t = torch.from_numpy(sample).cuda()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # recall against the exact FP64 K-NN on a sample of queries (outside the timed region)
    log("recall sample", len(sample))
    ex = oracle.search(Q[sample], X, w["metric"], L, K, exact=True)
    exv = ex["ex_v"]
    oracle_recall = float(oracle.recall_tie_aware(ex["top_v"], exv, True).mean())

    def sample_recall(idx):
        s64, _ = oracle.pair_scores(Q[sample], X, w["metric"], np.repeat(np.arange(len(sample)), K), idx.ravel())
        return float(oracle.recall_tie_aware(s64.reshape(-1, K), exv, True).mean())

    # rerank depth of the headline form: the smallest that keeps the method's own recall
    if args.compute == "fp32":
        head_rr = 0
    elif args.rerank == "auto":
        dbh = knn.Database(Xd, w["metric"], args.compute)
        for head_rr in (K, 2 * K, 4 * K):
            rec = sample_recall(dbh.search(Qd[sample_t], K, L, rerank=head_rr)[1].cpu().numpy())
            log(f"{args.compute} rerank {head_rr}: recall {rec:.4f} (oracle {oracle_recall:.4f})")
            if rec >= oracle_recall:
                break
        del dbh
        torch.cuda.empty_cache()
    else:
        head_rr = int(args.rerank)

    results = {}
    for comp in [args.compute] + [c for c in args.variants.split(",") if c and c != args.compute]:
        rr = 0 if comp == "fp32" else (head_rr if comp == args.compute else 4 * K)
        log("timing", comp, "rerank", rr)
        results[comp] = run_variant(knn, Xd, Qd, w, comp, rr, args.steps, args.warmup, sample_t)
    for comp, r in results.items():
        s64, _ = oracle.pair_scores(Q[sample], X, w["metric"], np.repeat(np.arange(len(sample)), K), r["idx_sample"].ravel())
        r["recall_at_10"] = float(oracle.recall(r["idx_sample"], ex["ex_i"]).mean())
        r["recall_at_10_tie_aware"] = float(oracle.recall_tie_aware(s64.reshape(-1, K), exv, True).mean())
        # returned values against the FP64 scores of the returned rows
        err = np.abs(r["val_sample"].astype(np.float64).ravel() - s64)
        r["max_score_abs_err"] = float(err.max())
        r["max_score_rel_err"] = float((err / np.maximum(np.abs(s64), 1e-30)).max())
        del r["idx_sample"], r["val_sample"]

    head = results[args.compute]
    flops = 2.0 * M * N * dpad(D, args.compute)
    line = {
        "metric": METRIC,
        "value": head["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.compute,
        "data": "synthetic (SIFT1M-shaped integer Gaussian mixture; no dataset)",
        "config": {"workload": name, "metric": w["metric"], "M": M, "N": N, "D": D, "K": K, "L": L,
                   "compute": args.compute, "rerank_k": head["rerank_k"]},
        "recall_at_10": head["recall_at_10"],
        "recall_at_10_tie_aware": head["recall_at_10_tie_aware"],
        "recall_sample_queries": len(sample),
        # the metric's condition, checked on the sample (integer data has exact ties at the
        # 10th distance, so the tie-aware recall of eq. recall-def is the one that decides)
        "recall_target_met": head["recall_at_10_tie_aware"] >= 0.95,
        "max_score_rel_err": head["max_score_rel_err"],
        "oracle_fp64_recall_at_10_tie_aware": oracle_recall,
        "roofline": {
            "bound": "mfma",
            "achieved": head["fused_tflops"],
            "peak": PEAK_TFLOPS[args.compute],
            "unit": "TFLOP/s",
            "frac": head["fused_frac_of_peak"],
            "traffic": measured_traffic(args.compute),
            "kernel": "fused distance GEMM + bin reduce",
            "kernel_ms": head["fused_kernel_ms"],
            "flops_per_launch": flops,
            # from the committed counter runs of this kernel (null once the sources change):
            # matrix-pipe busy fraction and the clock it ran at (the nominal peak assumes 2.4 GHz)
            "mfma_busy": _counter_figure(f"mfma_busy[{args.compute}]"),
            "est_clock_ghz": _counter_figure(f"est_clock_ghz[{args.compute}]"),
        },
        "variants": {k: v for k, v in results.items() if k != args.compute},
    }
    ck = line["roofline"]["est_clock_ghz"]
    if ck:  # the same rate against the peak at the clock the counters saw (peak assumes 2.4 GHz)
        line["roofline"]["frac_at_est_clock"] = head["fused_frac_of_peak"] * 2.4 / ck
    if line["roofline"]["traffic"] is not None:  # measured HBM bytes over the kernel's time
        line["roofline"]["traffic_gb_s"] = line["roofline"]["traffic"] / (head["fused_kernel_ms"] * 1e-3) / 1e9
    # context for the fraction of peak: a large square BF16 GEMM from the vendor library
    # (hipBLASLt through torch.matmul) on the same GPU, same nominal peak
    A = torch.randn((8192, 8192), device="cuda").to(torch.bfloat16)
    Bm = torch.randn((8192, 8192), device="cuda").to(torch.bfloat16)
    Cm = torch.empty((8192, 8192), device="cuda", dtype=torch.bfloat16)
    tg = time_kernel_events(lambda: torch.matmul(A, Bm, out=Cm), 20)
    line["roofline"]["library_gemm_bf16_8192_tflops"] = 2.0 * 8192 ** 3 / tg / 1e12
    del A, Bm, Cm
    torch.cuda.empty_cache()
    rows = [r for r in args.rows.split(",") if r]
    if "fp8_equal_recall" in rows and "fp32" in results:
        # FP8 + rerank at the FP32 form's recall: more bins (a bin's FP8 winner may be the
        # wrong row of the bin; smaller bins hold fewer rivals) and a deeper rerank
        target = results["fp32"]["recall_at_10_tie_aware"]
        pick = None
        db8 = knn.Database(Xd, w["metric"], "fp8")
        for L8, Kr8 in ((L, 40), (2 * L, 64), (2 * L, 100), (4 * L, 100), (8 * L, 160), (16 * L, 256)):
            idx8 = db8.search(Qd[sample_t], K, L8, rerank=Kr8)[1].cpu().numpy()
            s64, _ = oracle.pair_scores(Q[sample], X, w["metric"], np.repeat(np.arange(len(sample)), K), idx8.ravel())
            rec = float(oracle.recall_tie_aware(s64.reshape(-1, K), exv, True).mean())
            log(f"fp8 L={L8} rerank={Kr8}: recall {rec:.4f} (target {target:.4f})")
            pick = (L8, Kr8, rec)
            if rec >= target:
                break
        del db8
        torch.cuda.empty_cache()
        r8 = run_variant(knn, Xd, Qd, w, "fp8", pick[1], args.steps, args.warmup, sample_t, L=pick[0])
        del r8["idx_sample"], r8["val_sample"]
        r8["recall_at_10_tie_aware"] = pick[2]
        r8["target_recall"] = target
        line["fp8_equal_recall"] = r8
    if "exact_expectation_L" in rows:
        # the headline form at the smallest L whose exact expected recall with balanced bins
        # reaches 0.95 (eq. recall is a lower bound of that expectation; eq. l:approx's L
        # is the one above)
        Le = next(n_b for n_b in range(K, L + 1) if oracle.recall_exact_balanced(N, n_b, K) >= 0.95)
        exe = oracle.search(Q[sample], X, w["metric"], Le, K)
        re_ = run_variant(knn, Xd, Qd, w, args.compute, head_rr, args.steps, args.warmup, sample_t, L=Le)
        s64, _ = oracle.pair_scores(Q[sample], X, w["metric"], np.repeat(np.arange(len(sample)), K),
                                    re_["idx_sample"].ravel())
        re_["recall_at_10"] = float(oracle.recall(re_["idx_sample"], ex["ex_i"]).mean())
        re_["recall_at_10_tie_aware"] = float(oracle.recall_tie_aware(s64.reshape(-1, K), exv, True).mean())
        re_["oracle_fp64_recall_at_10_tie_aware"] = float(oracle.recall_tie_aware(exe["top_v"], exv, True).mean())
        re_["expected_recall_balanced_bins"] = oracle.recall_exact_balanced(N, Le, K)
        re_["expected_recall_paper_bound"] = oracle.recall_bound_paper(K, Le)
        del re_["idx_sample"], re_["val_sample"]
        line["exact_expectation_L"] = re_
    others = {}
    for name_r, fn in (("mips_small", lambda: row_mips_small(torch, knn, datagen)),
                       ("cosine_glove", lambda: row_cosine_glove(torch, knn, datagen, oracle, 5, 1)),
                       ("batched", lambda: row_batched(torch, knn, datagen, 3)),
                       ("mips_backward", lambda: row_mips_backward(torch, knn, datagen, 3)),
                       ("approx", lambda: row_approx(torch, knn, datagen)),
                       ("ablation", lambda: row_ablation(torch, knn, datagen))):
        if name_r in rows:
            log("workload", name_r)
            others[name_r] = fn()
            log(" ", json.dumps(others[name_r]))
    if others:
        line["other_workloads"] = others
    line["perf_model"] = perf_model_rows(line)
    if not args.no_cpu:
        threads = len(os.sched_getaffinity(0))
        log("cpu baseline: oracle on", threads, "threads")
        n0 = min(threads, 16)
        t0 = time.perf_counter()
        oracle.search(Q[:n0], X, w["metric"], L, K, nthreads=threads)
        per_q = max((time.perf_counter() - t0) / n0, 1e-4)
        S = int(min(M, max(8, args.cpu_seconds / per_q)))
        t0 = time.perf_counter()
        oracle.search(Q[:S], X, w["metric"], L, K, nthreads=threads)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": S / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
                                "sample": f"first {S} of the {M} queries against all {N} rows "
                                          f"(FP64 scores + bins + top-K), {dt:.1f} s"}
        # the exact ground truth beside it: a full sort of all N scores per query
        n1 = min(M, max(2 * threads, 16))
        t0 = time.perf_counter()
        oracle.search(Q[:n1], X, w["metric"], L, K, exact=True, nthreads=threads)
        dte = time.perf_counter() - t0
        line["cpu_baseline"]["exact_knn_value"] = n1 / dte
        line["cpu_baseline"]["exact_knn_sample"] = (f"first {n1} queries: FP64 scores, bins + top-K and a full "
                                                    f"sort of all {N} scores, {dte:.1f} s")
    if not line["recall_target_met"]:
        log(f"WARNING: sampled recall@10 {line['recall_at_10_tie_aware']:.4f} is below 0.95: the headline "
            "value does not meet the metric's recall condition")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
