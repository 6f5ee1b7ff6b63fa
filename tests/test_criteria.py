"""The paper's four performance criteria and its size fit (section IV.A,
Tables 3 and 5, Fig. 1): the measurement helper reproduces every printed
figure from the paper's own times, peaks and counts."""
import json
import os

import pytest

from paper_1004_1680_amd import criteria as C

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table5_criteria.json")))


def test_counts_give_the_paper_totals():
    ops = GOLD["op_counts"]
    assert C.PAPER_FLOP_PER_CELL_STEP == sum(ops.values())
    fl = GOLD["floats"]
    reads = (fl["cfl_read"] + fl["fluid_updates"] * fl["fluid_read"]
             + fl["magnetic_updates"] * fl["magnetic_read"] + fl["transposes"] * fl["transpose_read"])
    writes = (fl["fluid_updates"] * fl["fluid_write"] + fl["magnetic_updates"] * fl["magnetic_write"]
              + fl["transposes"] * fl["transpose_write"])
    assert C.PAPER_FLOATS_PER_CELL_STEP == reads + writes
    # the totals are printed in units of 2^30
    cells, gib = 128 ** 3, 2 ** 30
    tot = GOLD["totals_128"]
    assert round(C.PAPER_FLOP_PER_CELL_STEP * cells / gib, 2) == tot["gflop"]
    assert round(4 * C.PAPER_FLOATS_PER_CELL_STEP * cells / gib, 2) == tot["gbytes"]
    assert round(4 * reads * cells / gib, 2) == tot["gbytes_read"]
    assert round(4 * writes * cells / gib, 2) == tot["gbytes_write"]


@pytest.mark.parametrize("arch", list(GOLD["table5"]["columns"]))
def test_table5_is_reproduced(arch):
    t5 = GOLD["table5"]
    col = t5["columns"][arch]
    ref = t5["columns"][t5["ref"]]
    cells = t5["n"] ** 3
    args = (col["time_ms"], ref["time_ms"], cells, col["peak_gflops"], col["peak_gbs"], ref["peak_gflops"])
    # the printed fractions divide the rounded totals (4.62 and 2.23, in
    # units of 2^30) by the times
    tot = GOLD["totals_128"]
    c = C.criteria(*args, flop_per_cell=tot["gflop"] * 2 ** 30 / cells,
                   bytes_per_cell=tot["gbytes"] * 2 ** 30 / cells, giga=2 ** 30)
    assert round(c["code_speedup"], 1) == col["code_speedup"]
    assert abs(c["fractional_speedup"] - col["fractional_speedup"]) <= 0.005 + 1e-12
    assert round(100 * c["flops_fraction"], 1) == col["flops_pct"]
    assert round(100 * c["bandwidth_fraction"], 1) == col["bandwidth_pct"]
    # the exact counts land within a tenth of a percentage point
    e = C.criteria(*args, giga=2 ** 30)
    assert abs(100 * e["flops_fraction"] - col["flops_pct"]) <= 0.1
    assert abs(100 * e["bandwidth_fraction"] - col["bandwidth_pct"]) <= 0.1


def test_decimal_units_raise_the_fractions_by_2_30_over_1e9():
    c2 = C.criteria(83, None, 128 ** 3, 748.8, 141, None, giga=2 ** 30)
    c10 = C.criteria(83, None, 128 ** 3, 748.8, 141, None)
    assert c10["code_speedup"] is None and c10["fractional_speedup"] is None
    assert c10["flops_fraction"] / c2["flops_fraction"] == pytest.approx(2 ** 30 / 1e9, rel=1e-12)
    assert c10["bandwidth_fraction"] / c2["bandwidth_fraction"] == pytest.approx(2 ** 30 / 1e9, rel=1e-12)


def test_table3_speedups_and_slope():
    t3 = GOLD["table3"]
    for t1, tg, s in zip(t3["x86_1_ms"], t3["cuda_ms"], t3["speedup"]):
        c = C.criteria(tg, t1, 1, 1, 1, None)
        assert round(c["code_speedup"], 1) == s
    # one core is N^3 work throughout: slope near 3 (endpoints alone: 2.98)
    assert 2.95 <= C.size_slope(t3["n"], t3["x86_1_ms"]) <= 3.0
    # the GPU column is launch- and occupancy-limited at small n: well below 3
    assert C.size_slope(t3["n"], t3["cuda_ms"]) < 2.5


def test_slope_of_power_laws():
    ns = [16, 32, 48, 64, 96, 128]
    for p in (1.0, 2.0, 3.0):
        assert C.size_slope(ns, [0.37 * n ** p for n in ns]) == pytest.approx(p, abs=1e-12)
    with pytest.raises(ValueError):
        C.size_slope([64], [1.0])
    with pytest.raises(ValueError):
        C.size_slope([64, 64], [1.0, 2.0])


def test_host_core_peak(tmp_path):
    info = tmp_path / "cpuinfo"
    info.write_text("model name\t: Test CPU\nflags\t\t: fpu sse2 avx2 avx512f\ncpu MHz\t\t: 1500.0\n"
                    "model name\t: Test CPU\ncpu MHz\t\t: 2000.0\n")
    g, desc = C.host_core_peak_gflops(str(info), str(tmp_path / "none"))
    assert g == pytest.approx(2.0 * 2 * 16 * 2)
    assert "Test CPU" in desc
    info.write_text("model name\t: Old CPU\nflags\t\t: fpu sse2 avx2\ncpu MHz\t\t: 3000.0\n")
    g, _ = C.host_core_peak_gflops(str(info), str(tmp_path / "none"))
    assert g == pytest.approx(3.0 * 2 * 8 * 2)
    g, _ = C.host_core_peak_gflops(str(tmp_path / "missing"), str(tmp_path / "none"))
    assert g is None
