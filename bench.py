#!/usr/bin/env python3
"""Throughput of the approximate K-NN search on one MI355X.

Workload (default): relaxed-L2 search, M = 10,000 queries against N = 1,000,000 rows,
D = 128, K = 10, L = 176 bins (the smallest L with ((L-1)/L)^(K-1) >= 0.95), on
SIFT1M-shaped synthetic data (integers in [0, 255] from a 256-centre Gaussian mixture).

One step = one pass of the hot path over the whole query batch, inputs resident in
HBM: query preparation + distance GEMM with the bin-reduce epilogue + top-K select
(+ FP32 rerank of the best `--rerank` bin winners for the BF16 / FP8 forms).  The
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


def run_variant(knn, Xd, Qd, w, compute, rerank, steps, warmup, sample_idx):
    import torch
    M, N, D, K, L = Qd.shape[0], Xd.shape[0], w["D"], w["K"], w["L"]
    t0 = time.perf_counter()
    db = knn.Database(Xd, w["metric"], compute)
    prep_s = time.perf_counter() - t0
    out = (torch.empty((M, K), dtype=torch.float32, device="cuda"), torch.empty((M, K), dtype=torch.int32, device="cuda"))

    def step():
        db.search(Qd, K, L, rerank=rerank, out=out)

    sec = time_steps(step, steps, warmup)
    # the distance + bin-reduce kernel alone, on prepared queries
    qbuf = db.prepare_queries(Qd)
    bins = (torch.empty((M, L), dtype=torch.float32, device="cuda"), torch.empty((M, L), dtype=torch.int32, device="cuda"))
    ksec = time_kernel_events(lambda: db.partial_reduce(qbuf, M, L, out=bins, resolve=False), max(steps, 5))
    flops = 2.0 * M * N * dpad(D, compute)
    res = {
        "compute": compute,
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
    del db, qbuf, bins
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--compute", default="bf16", choices=["fp32", "bf16", "fp8"], help="headline compute type")
    ap.add_argument("--rerank", type=int, default=40, help="bin winners rescored in FP32 (low-precision forms)")
    ap.add_argument("--variants", default="fp32,fp8", help="other compute types to time next to the headline")
    ap.add_argument("--recall-sample", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a known-size kernel for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md on sharding); "
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

    results = {}
    for comp in [args.compute] + [c for c in args.variants.split(",") if c and c != args.compute]:
        rr = 0 if comp == "fp32" else args.rerank
        log("timing", comp, "rerank", rr)
        results[comp] = run_variant(knn, Xd, Qd, w, comp, rr, args.steps, args.warmup, sample_t)

    # recall against the exact FP64 K-NN on a sample of queries (outside the timed region)
    log("recall sample", len(sample))
    ex = oracle.search(Q[sample], X, w["metric"], L, K, exact=True)
    kth = ex["ex_v"][:, -1]
    for comp, r in results.items():
        s64, _ = oracle.pair_scores(Q[sample], X, w["metric"], np.repeat(np.arange(len(sample)), K), r["idx_sample"].ravel())
        r["recall_at_10"] = float(oracle.recall(r["idx_sample"], ex["ex_i"]).mean())
        r["recall_at_10_tie_aware"] = float(oracle.recall_tie_aware(s64.reshape(-1, K), kth, True).mean())
        del r["idx_sample"], r["val_sample"]
    oracle_recall = float(oracle.recall_tie_aware(ex["top_v"], kth, True).mean())

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
        "oracle_fp64_recall_at_10_tie_aware": oracle_recall,
        "roofline": {
            "bound": "mfma",
            "achieved": head["fused_tflops"],
            "peak": PEAK_TFLOPS[args.compute],
            "unit": "TFLOP/s",
            "frac": head["fused_frac_of_peak"],
            "traffic": None,
            "kernel": "fused distance GEMM + bin reduce",
            "kernel_ms": head["fused_kernel_ms"],
            "flops_per_launch": flops,
        },
        "variants": {k: v for k, v in results.items() if k != args.compute},
    }
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
