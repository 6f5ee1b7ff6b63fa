"""bench.py's command line without a GPU: a request for more than one GPU
is refused with a message (the path runs on one GPU) before anything loads."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_power_sampler_reads_microwatts(tmp_path):
    import time
    sys.path.insert(0, ROOT)
    import bench
    f = tmp_path / "power1_average"
    f.write_text("250000000\n")                      # 250 W in microwatts
    ps = bench.PowerSampler(object(), period=0.001)  # no device: nothing found
    assert ps.path is None and ps.result(1.0, 1, 1) is None
    ps.path = str(f)
    with ps:
        time.sleep(0.02)
    r = ps.result(2.0, 4, 10 ** 9)
    assert r["samples"] >= 1 and r["avg_W"] == 250.0
    assert r["J_per_step"] == 125.0                  # 250 W x 2 s / 4 steps
    assert r["Mcell_updates_per_J"] == 8.0           # 4e9 cell-updates / 500 J


def test_cpu_baseline_reports_median_model_and_threads():
    sys.path.insert(0, ROOT)
    import bench
    out = bench.cpu_baseline({"n": 16, "ic": "orszag_tang"})
    assert out["kind"] == "oracle" and out["value"] > 0
    assert "median of 3 full steps" in out["sample"] and "the same initial state at 16^3" in out["sample"]
    model, threads, avail = bench.cpu_info()
    assert out["cores"] == threads >= 1 and out["cpu_model"] == model
    assert out["single_thread"]["cores"] == 1


def test_step_launch_names_are_the_profilers():
    """the kernel names bench.py looks up in a traffic summary (every launch
    of a step, each workload's launch mix) are those the profiler printed in
    the committed 512^3 summary"""
    import re
    sys.path.insert(0, ROOT)
    import bench
    text = open(os.path.join(ROOT, "profiles", "sweeps_ot512_fp32_hbm_traffic.md")).read()
    names = set(re.findall(r"^traffic_bytes\[([^\]@]+?)\]", text, re.M))

    class S:
        def chunk(self, d): return 256
        def pair_chunk(self, d): return 256
        def launch(self, k): return 512

    for fused, middle in ((True, True), (True, False)):
        for name, _ in bench.step_launches(S(), 512, 4, fused, "true", 0, middle):
            assert name in names, name
