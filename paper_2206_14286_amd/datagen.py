"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the search's arithmetic.
Both the HIP path's tests/benchmark and the CPU oracle take their inputs from here.

Stand-ins (no dataset is available or reproduced):
  * SIFT1M-shaped (App. A.5, Table 2, Euclidean): integer entries in [0, 255] drawn
    from a Gaussian mixture of ``centres`` centres (centres uniform integers in
    [0, 255]^D, sigma 20, rounded and clipped);
  * GloVe-1.2M-shaped (Table 2, cosine, D = 100 padded to 128 by the search):
    rows from a mixture of ``centres`` N(0, I) centres plus 0.5 N(0, I) noise,
    unit-normalised;
  * plain i.i.d. standard normal (MIPS).
Rows are emitted in draw order, never sorted by cluster: the recall model of
Sec. 5.1 assumes the positions of the true neighbours are uniformly random.

Seeds: numpy PCG64; stream ``seed`` for the database, ``seed + 1`` for the
queries, ``seed + 2`` for targets and batch sizes.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def normal(n: int, d: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """i.i.d. N(0, scale^2) rows, float32."""
    out = _rng(seed).standard_normal((n, d), dtype=np.float32)
    if scale != 1.0:
        out *= np.float32(scale)
    return out


def normal_device(n: int, d: int, seed: int, scale: float = 1.0, dtype=None, device: str = "cuda"):
    """i.i.d. N(0, scale^2) rows drawn on the device with torch's seeded generator: for
    inputs of many GB (the batched and backward workloads); the parity tests copy them back
    to the host to check sampled outputs against the oracle."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.randn((n, d), generator=g, device=device, dtype=torch.float32)
    if scale != 1.0:
        out.mul_(scale)
    return out if dtype is None else out.to(dtype)


def int_mixture(n: int, d: int, seed: int, centres: int = 256, sigma: float = 20.0,
                centre_seed: int = 12345) -> np.ndarray:
    """Integer-valued rows in [0, 255]: clip(round(mu_c + sigma * eps)), c uniform.

    The centres come from their own stream so that queries and database share them."""
    mu = _rng(centre_seed).integers(0, 256, size=(centres, d)).astype(np.float32)
    r = _rng(seed)
    c = r.integers(0, centres, size=n)
    out = np.empty((n, d), np.float32)
    step = 1 << 16
    for s in range(0, n, step):
        e = min(n, s + step)
        x = mu[c[s:e]] + np.float32(sigma) * r.standard_normal((e - s, d), dtype=np.float32)
        out[s:e] = np.clip(np.rint(x), 0, 255)
    return out


def unit_mixture(n: int, d: int, seed: int, centres: int = 1000, noise: float = 0.5,
                 centre_seed: int = 54321) -> np.ndarray:
    """Unit-norm rows: (mu_c + noise * eps) / |.|, centres N(0, I)."""
    mu = _rng(centre_seed).standard_normal((centres, d), dtype=np.float32)
    r = _rng(seed)
    c = r.integers(0, centres, size=n)
    out = np.empty((n, d), np.float32)
    step = 1 << 16
    for s in range(0, n, step):
        e = min(n, s + step)
        x = mu[c[s:e]] + np.float32(noise) * r.standard_normal((e - s, d), dtype=np.float32)
        nrm = np.sqrt((x.astype(np.float64) ** 2).sum(axis=1))
        out[s:e] = (x / np.where(nrm > 0, nrm, 1.0)[:, None]).astype(np.float32)
    return out


def batch_sizes(count: int, seed: int, lo: int = 1, hi: int = 4096) -> np.ndarray:
    """Log-uniform integer batch sizes in [lo, hi]: round(exp(U(ln lo, ln hi)))."""
    u = _rng(seed).uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


def targets(m: int, k: int, seed: int) -> np.ndarray:
    """Uniform random target positions in [0, k) (one per query)."""
    return _rng(seed).integers(0, k, size=m).astype(np.int64)


def score_matrix(rows: int, cols: int, seed: int, kind: str = "normal") -> np.ndarray:
    """float32 score matrices for the approx_max_k op on its own:
    'normal' i.i.d. N(0, 1); 'ints' integers in [-8, 8] (many exact ties); 'zeros' +0 and
    -0 in equal parts with a few +-1 (ties between the two zeros); 'masked' N(0, 1) with
    about a quarter of the entries set to -inf (masked-out scores)."""
    r = _rng(seed)
    if kind == "normal":
        return r.standard_normal((rows, cols), dtype=np.float32)
    if kind == "ints":
        return r.integers(-8, 9, size=(rows, cols)).astype(np.float32)
    if kind == "zeros":
        out = np.where(r.random((rows, cols)) < 0.5, np.float32(0.0), np.float32(-0.0)).astype(np.float32)
        pick = r.random((rows, cols))
        out[pick < 0.01] = 1.0
        out[pick > 0.99] = -1.0
        return out
    if kind == "masked":
        out = r.standard_normal((rows, cols), dtype=np.float32)
        out[r.random((rows, cols)) < 0.25] = -np.inf
        return out
    raise KeyError(kind)


# The shape of the paper's comparison of the fused op with a dense GEMM followed by a
# reshape and an argmax per bin (appendix on the alternative implementation):
# queries 1024 x 128, database 2^20 x 128, L = 128 bins of 8192 rows, FP32, MIPS.
ABLATION = dict(M=1024, N=1 << 20, D=128, L=128)

# Databases of the batched workload: (N, D), BF16 N(0, 1) rows, MIPS, K = 10
BATCHED_DBS = [(100_000, 64), (1_000_000, 96), (4_000_000, 128), (16_000_000, 256)]
BATCHED_COUNT = 256

# The single-database workloads: (metric, M, N, D, K, L, description)
WORKLOADS = {
    "mips_small": dict(metric="mips", M=64, N=65536, D=128, K=10, L=2048,
                       data="iid N(0,1) fp32"),
    "l2_sift": dict(metric="l2", M=10000, N=1000000, D=128, K=10, L=176,
                    data="integers in [0,255], 256-centre Gaussian mixture, sigma 20"),
    "cosine_glove": dict(metric="cosine", M=10000, N=1200000, D=100, K=100, L=16384,
                         data="unit rows, 1000-centre Gaussian mixture"),
    "mips_backward": dict(metric="mips", M=8192, N=4000000, D=256, K=64, L=32768,
                          data="bf16 N(0,1)/sqrt(D)"),
}


def make(name: str, seed: int = 0, M: int | None = None, N: int | None = None):
    """Queries and database of a named workload (optionally with fewer queries or rows)."""
    w = WORKLOADS[name]
    M = w["M"] if M is None else M
    N = w["N"] if N is None else N
    D = w["D"]
    if name == "mips_small":
        return normal(M, D, seed + 1), normal(N, D, seed)
    if name == "l2_sift":
        return int_mixture(M, D, seed + 1), int_mixture(N, D, seed)
    if name == "cosine_glove":
        return unit_mixture(M, D, seed + 1), unit_mixture(N, D, seed)
    if name == "mips_backward":
        s = 1.0 / math.sqrt(D)
        return normal(M, D, seed + 1, s), normal(N, D, seed, s)
    raise KeyError(name)
