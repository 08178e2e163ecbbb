"""The accelerator performance model of Sec. 4 applied to MI355X.

eq. roofline bounds a kernel's FLOP rate by three ceilings: the matrix peak pi, memory
bandwidth times memory intensity (beta * I_MEM, Sec. 4.2), and the coefficient-wise
operation (COP) rate times COP intensity (gamma * I_COP, Sec. 4.3, eq. pr:icop with
I_COP = 2D / C for C COPs per score).  For the bin-reduce kernel the paper estimates
the memory intensity from its transfers (Sec. 5, eq. for I_MEM): the queries once, the
database once per query block of ib queries, and the M x L outputs (value and index).

MI355X figures: dense matrix peaks (FP32 157.3, BF16 2516.6, FP8 5033.2 TFLOP/s), HBM3E
8 TB/s, and gamma = 256 CUs x 64 lanes x 2.4 GHz = 39.32 T lane-operations/s (a compare
or a select is one lane-operation per score).
"""
from __future__ import annotations

MI355X = {"pi_tflops": {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}, "beta_gbs": 8000.0,
          "gamma_tcops": 256 * 64 * 2.4e9 / 1e12}
ELEM_BYTES = {"fp32": 4, "bf16": 2, "fp8": 1}


def cops_per_score(metric: str) -> int:
    """C of the bin-reduce kernel as the paper counts it on any chip: a compare and two
    conditional moves per score (Algorithm 1), plus one subtraction for the relaxed L2
    distance (appendix on Euclidean search).  The TPU-only terms of Table 2 (masking a
    non-power-of-two N, broadcasting the half norms) are not costs on MI355X."""
    return 3 + (1 if metric == "l2" else 0)


def cop_intensity(D: int, C: float) -> float:
    """eq. pr:icop: I_COP = 2D / C."""
    return 2.0 * D / C


def cop_budget(D: int, pi_tflops: float, gamma_tcops: float) -> float:
    """eq. c-limit: the largest C that keeps gamma * I_COP at or above pi, C = 2 D gamma / pi."""
    return 2.0 * D * gamma_tcops / pi_tflops


def mem_intensity(M: int, N: int, D: int, L: int, elem_bytes: float, ib: int) -> float:
    """FLOPs per byte of the bin-reduce kernel: 2MND over the transfers of the queries
    (M D elements), the database once per block of ib queries (N D M / ib elements) and
    the outputs (2 x 4 bytes per bin)."""
    return 2.0 * M * N * D / (elem_bytes * (M * D + N * D * M / ib) + 8.0 * M * L)


def ceiling(pi_tflops: float, beta_gbs: float, gamma_tcops: float, i_mem: float, i_cop: float):
    """eq. roofline: (attainable GFLOP/s, which ceiling binds: 'matrix', 'memory' or 'cop')."""
    c = {"matrix": pi_tflops * 1e3, "memory": beta_gbs * i_mem, "cop": gamma_tcops * 1e3 * i_cop}
    bound = min(c, key=c.get)
    return c[bound], bound


# The distance kernel's own least VALU work per score (it folds each group of 4 scores
# into the running bin winner with two 3-input maxima, a compare and a select): one
# lane-operation per score.  Where no counter run measured the kernel's C, this lower
# bound of C gives an upper bound of the COP ceiling, so the ceiling still bounds it.
C_KERNEL_MIN = 1.0


def entry(name: str, compute: str, metric: str, M: int, N: int, D: int, L: int, ib: int,
          measured_tflops: float, hbm_bytes: float | None = None, measured_c: float | None = None,
          clock_ghz: float | None = None, chip: dict = MI355X) -> dict:
    """One row of the Table 2 layout for a measured launch of the bin-reduce kernel.

    Two ceilings of eq. roofline are given: the paper's (its C for Algorithm 1, its
    transfer estimate I_MEM with the database read once per query block of ib queries,
    the nominal 2.4 GHz clock) as context, and the kernel's, which is the one the measured
    rate is held to (frac_of_ceiling): C is the kernel's own (measured from instruction
    counters where available, else C_KERNEL_MIN), I_MEM comes from the measured traffic
    where available, else from the algorithmic bytes, and the matrix and COP rates are
    scaled to the clock the counters saw where that is known (the chip lowers its clock
    under load, and its dense peak assumes 2.4 GHz)."""
    pi = chip["pi_tflops"][compute]
    C = cops_per_score(metric)
    i_cop = cop_intensity(D, C)
    i_mem = mem_intensity(M, N, D, L, ELEM_BYTES[compute], ib)
    flops = 2.0 * M * N * D
    i_mem_meas = flops / hbm_bytes if hbm_bytes else None
    g_paper, bound_paper = ceiling(pi, chip["beta_gbs"], chip["gamma_tcops"], i_mem_meas or i_mem, i_cop)
    f = (clock_ghz / 2.4) if clock_ghz else 1.0
    c_k = measured_c if measured_c else C_KERNEL_MIN
    # the kernel's memory ceiling: its measured traffic, else the least it can move (every
    # input once and the bins out), which bounds it whatever the caches reuse
    i_mem_alg = mem_intensity(M, N, D, L, ELEM_BYTES[compute], M)
    g, bound = ceiling(pi * f, chip["beta_gbs"], chip["gamma_tcops"] * f, i_mem_meas or i_mem_alg,
                       cop_intensity(D, c_k))
    return {"workload": name, "compute": compute, "D": D, "N": N, "M": M, "L": L,
            "C_paper": C, "I_COP_paper": round(i_cop, 1), "ceiling_gflops_paper": round(g_paper),
            "bound_paper": bound_paper,
            "C_kernel": c_k, "C_kernel_measured": measured_c is not None, "clock_ghz": clock_ghz or 2.4,
            "clock_measured": clock_ghz is not None,
            "I_MEM": round(i_mem, 1), "I_MEM_algorithmic": round(i_mem_alg, 1),
            "I_MEM_measured": round(i_mem_meas, 1) if i_mem_meas else None,
            "I_COP": round(cop_intensity(D, c_k), 1), "ceiling_gflops": round(g), "bound": bound,
            "measured_gflops": round(measured_tflops * 1e3), "frac_of_ceiling": measured_tflops * 1e3 / g}


def entry_memory(name: str, flops: float, hbm_bytes: float, seconds: float, chip: dict = MI355X) -> dict:
    """A row for a kernel bound by memory traffic alone (the backward's gathers and
    scatter-adds): eq. roofline with I_MEM = FLOP / algorithmic bytes; the matrix and COP
    ceilings are far above it."""
    i_mem = flops / hbm_bytes
    g = chip["beta_gbs"] * i_mem
    return {"workload": name, "compute": "fp32", "I_MEM": round(i_mem, 3), "ceiling_gflops": round(g, 1),
            "bound": "memory", "measured_gflops": round(flops / seconds / 1e9, 1),
            "frac_of_ceiling": flops / seconds / 1e9 / g}
