"""bench.py's size sweep end to end on the GPU (small sizes): one JSON line
with a record per size, the criteria of each, the slope fit, and a markdown
summary made from it."""
import json
import os
import subprocess
import sys

import pytest

from paper_1004_1680_amd import criteria as C

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_size_sweep_small():
    print("case: bench.py --size-sweep 16,32", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--size-sweep", "16,32",
                        "--no-cpu", "--no-tune", "--sweep-seconds", "0.02"],
                       capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["higher_is_better"] is False and d["n_gpus"] == 1
    ss = d["size_sweep"]
    assert [x["n"] for x in ss["sizes"]] == [16, 32]
    for x in ss["sizes"]:
        assert x["steps"] >= 10 and x["ms_per_step"] > 0
        assert x["mcell_s"] == pytest.approx(x["n"] ** 3 / (x["ms_per_step"] * 1e3), rel=1e-9)
        c = x["criteria"]
        assert c["code_speedup"] is None          # no one-thread oracle with --no-cpu
        assert c["gflops"] == pytest.approx(C.PAPER_FLOP_PER_CELL_STEP * x["n"] ** 3
                                            / (x["ms_per_step"] * 1e-3) / 1e9, rel=1e-9)
    assert ss["slope_all"] == pytest.approx(C.size_slope([16, 32], [x["ms_per_step"] for x in ss["sizes"]]))
    assert ss["slope_large"] is None              # no size >= 128
    md = C.markdown(ss)
    assert md.count("\n| 16 |") == 1 and md.count("\n| 32 |") == 1
