"""The oracle's performance-model formulas against the values the paper prints.

Fixture: tests/golden/paper_tables.json (Table 1, Table 2, and the COP budgets the
text states after eq. c-limit).  A dropped factor of 2 in eq. c-limit or eq. pr:icop,
or a swapped beta/gamma term in eq. roofline, fails one of these."""
import json
import math
import os

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
G = json.load(open(os.path.join(HERE, "golden", "paper_tables.json")))


def test_cop_budgets_stated_after_c_limit():
    t1 = G["table1"]
    for chip, budget in G["cop_budget_D128"].items():
        if chip.startswith("_"):
            continue
        c = oracle.cop_budget(128, t1[chip]["pi"], t1[chip]["gamma"])
        # the text quotes the budget as a whole number of COPs
        assert math.floor(c + 1e-9) == budget, (chip, c)


def test_table2_cop_intensity():
    for name, row in G["table2"].items():
        assert round(oracle.cop_intensity(row["D"], row["C"]), 1) == row["I_COP"], name


def test_table2_measurements_under_the_roofline():
    t1 = G["table1"]
    for name, row in G["table2"].items():
        for chip, key in (("TPU V3", "gflops_tpu_v3"), ("TPU V4", "gflops_tpu_v4")):
            h = t1[chip]
            ceil = oracle.roofline_gflops(h["pi"], h["beta"], h["gamma"], row["I_MEM"],
                                          oracle.cop_intensity(row["D"], row["C"]))
            assert row[key] <= ceil, (name, chip, row[key], ceil)
            # every measurement is within 40 % of its ceiling (the paper's point: near peak)
            assert row[key] >= 0.6 * ceil, (name, chip, row[key], ceil)


def test_sift_on_v4_is_the_cop_bound_case():
    # Table 2's Sift run on TPU V4 is the one limited by COPs (C = 6 > the budget of 4)
    h = G["table1"]["TPU V4"]
    row = G["table2"]["Sift1M"]
    cop = h["gamma"] * 1e3 * oracle.cop_intensity(row["D"], row["C"])
    assert cop < h["pi"] * 1e3
    assert oracle.roofline_gflops(h["pi"], h["beta"], h["gamma"], row["I_MEM"],
                                  oracle.cop_intensity(row["D"], row["C"])) == cop
    assert row["C"] > oracle.cop_budget(row["D"], h["pi"], h["gamma"])


# ---------------------------------------------------------------- the product's model
def test_product_perf_model_reproduces_the_paper():
    """The performance model that the benchmark reports (paper_2206_14286_amd.perf_model)
    gives Table 2's COP intensities, the two COP budgets stated after eq. c-limit, and,
    with Table 1's chips, ceilings that Table 2's measured TPU rates do not exceed, with
    Sift on TPU V4 bound by COPs; it agrees with the oracle's formulas."""
    from paper_2206_14286_amd import perf_model as pm
    g = G
    t1, t2 = g["table1"], g["table2"]
    for ds in t2.values():
        assert abs(pm.cop_intensity(ds["D"], ds["C"]) - ds["I_COP"]) < 0.05
        assert pm.cop_intensity(ds["D"], ds["C"]) == oracle.cop_intensity(ds["D"], ds["C"])
    for chip, want in g["cop_budget_D128"].items():
        if chip.startswith("_"):
            continue
        c = t1[chip]
        assert round(pm.cop_budget(128, c["pi"], c["gamma"])) == want
    for chip, col in (("TPU V3", "gflops_tpu_v3"), ("TPU V4", "gflops_tpu_v4")):
        c = t1[chip]
        for ds in t2.values():
            gf, bound = pm.ceiling(c["pi"], c["beta"], c["gamma"], ds["I_MEM"], ds["I_COP"])
            assert gf == oracle.roofline_gflops(c["pi"], c["beta"], c["gamma"], ds["I_MEM"], ds["I_COP"])
            assert ds[col] <= gf * 1.0001
    c = t1["TPU V4"]
    assert pm.ceiling(c["pi"], c["beta"], c["gamma"], t2["Sift1M"]["I_MEM"], t2["Sift1M"]["I_COP"])[1] == "cop"
    # MI355X: the BF16 matrix peak is exactly at the COP ceiling for L2 at D = 128 (C = 4)
    m = pm.MI355X
    assert abs(pm.cop_budget(128, m["pi_tflops"]["bf16"], m["gamma_tcops"]) - 4.0) < 0.01
