"""Host-side parts of bench.py (no GPU): the one-GPU guard, the reader of the committed
counter summary (figures only while the kernel sources hash to the recorded value), and
the performance-model rows built from a bench line."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _summary(tmp_path, sha):
    p = tmp_path / "counters.md"
    p.write_text("# summary\n\n"
                 f"- source_sha256: {sha}\n"
                 "- traffic_bytes_per_launch[bf16]: 123456789\n"
                 "- valu_ops_per_score[bf16]: 1.500\n"
                 "- est_clock_ghz[bf16]: 1.80\n")
    return str(p)


def test_counter_figures_follow_the_source_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS_FILE", _summary(tmp_path, bench.kernel_source_digest()))
    assert bench.measured_traffic("bf16") == 123456789.0
    assert bench.measured_cops("bf16") == 1.5
    assert bench._counter_figure("est_clock_ghz[bf16]") == 1.8
    assert bench.measured_traffic("fp8") is None  # not recorded
    monkeypatch.setattr(bench, "COUNTERS_FILE", _summary(tmp_path, "0" * 64))  # other sources
    assert bench.measured_traffic("bf16") is None
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("bf16") is None


def test_committed_summary_is_readable():
    """The committed summary names a hash and the figures bench.py reads, for every form."""
    text = open(bench.COUNTERS_FILE).read()
    assert "- source_sha256:" in text
    for comp in ("bf16", "fp8", "fp32"):
        for key in ("traffic_bytes_per_launch", "valu_ops_per_score", "mfma_busy", "est_clock_ghz"):
            assert f"- {key}[{comp}]:" in text


def test_perf_model_rows_from_a_bench_line(monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS_FILE", "/nonexistent")
    line = {"dtype": "bf16", "config": {"M": 10000, "N": 1000000, "D": 128, "L": 176},
            "roofline": {"achieved": 1400.0},
            "variants": {"fp32": {"fused_tflops": 127.0, "L": 176}}}
    rows = bench.perf_model_rows(line)
    assert [r["compute"] for r in rows] == ["bf16", "fp32"]
    bf16, fp32 = rows
    # Sec. 4 with the paper's C = 4 for L2: I_COP = 2D/C = 64, so the COP ceiling equals
    # the matrix peak (gamma * 64 = 2.52 PFLOP/s); the paper's transfer estimate (the
    # database read once per 256-query block) puts the memory ceiling below both
    assert bf16["I_COP_paper"] == pytest.approx(64.0)
    i_mem = 2.0 * 10000 * 1000000 * 128 / (2 * (10000 * 128 + 1000000 * 128 * 10000 / 256) + 8 * 10000 * 176)
    assert bf16["I_MEM"] == pytest.approx(i_mem, rel=1e-3)
    assert bf16["ceiling_gflops_paper"] == pytest.approx(min(2516600, 8000 * i_mem), rel=1e-3)
    assert bf16["bound_paper"] == "memory"
    # the kernel's ceiling: without counters, C is the kernel's least (1 per score) and
    # the clock nominal, so the matrix peak binds
    assert bf16["C_kernel"] == 1.0 and not bf16["C_kernel_measured"] and bf16["bound"] == "matrix"
    assert fp32["bound"] == "matrix"
    assert fp32["ceiling_gflops"] == pytest.approx(157300, rel=1e-6)
    assert bf16["frac_of_ceiling"] == pytest.approx(1400e3 / bf16["ceiling_gflops"])
    assert bf16["I_MEM_measured"] is None  # no counters for these sources


def test_perf_model_uses_the_counter_clock_and_measured_c(tmp_path, monkeypatch):
    """With a counter summary for the current sources the kernel's ceiling takes the
    measured C and the measured clock: the matrix peak scales by clock / 2.4 GHz."""
    monkeypatch.setattr(bench, "COUNTERS_FILE", _summary(tmp_path, bench.kernel_source_digest()))
    line = {"dtype": "bf16", "config": {"M": 10000, "N": 1000000, "D": 128, "L": 176},
            "roofline": {"achieved": 1400.0}, "variants": {}}
    (row,) = bench.perf_model_rows(line)
    assert row["C_kernel"] == 1.5 and row["C_kernel_measured"] and row["clock_ghz"] == 1.8
    assert row["ceiling_gflops"] == pytest.approx(2516600 * 1.8 / 2.4, rel=1e-3)
    assert row["I_MEM_measured"] == pytest.approx(2.0 * 10000 * 1000000 * 128 / 123456789, rel=1e-3)


def _committed_bench_lines():
    """Bench lines recorded under profiles/ (a JSON line after a '```json' fence)."""
    import glob
    import json
    out = []
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "bench_*.md"))):
        text = open(f).read()
        if "```json" in text:
            out.append((f, json.loads(text.split("```json", 1)[1].split("```", 1)[0])))
    return out


def test_committed_bench_lines_stay_under_their_ceilings(monkeypatch):
    """Every performance-model row of a committed bench line, and the rows the current
    model derives from that line's measurements, has frac_of_ceiling <= 1: the kernel's
    ceiling (its own C, the clock the counters saw) bounds every measured launch."""
    lines = _committed_bench_lines()
    assert lines, "no bench line recorded under profiles/"
    for f, line in lines:
        for r in line["perf_model"]:
            assert r["frac_of_ceiling"] <= 1.0, (f, r["workload"], r["compute"], r["frac_of_ceiling"])
        for r in bench.perf_model_rows(line):
            assert r["frac_of_ceiling"] <= 1.0, (f, r["workload"], r["compute"], r["frac_of_ceiling"])
