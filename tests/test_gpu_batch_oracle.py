"""Batched ensembles against the FP64 oracle, and the 64-box benchmark
ensemble over 100 steps.

Every box of an uneven ensemble, advanced from a captured HIP graph with its
own device-side CFL step, is compared element by element with the oracle
run of the same box (oracle.run: the CFL condition before each step, then
F_x M_x F_y M_y F_z M_z M_z F_z M_y F_y M_x F_x, section II.B) at the
tier's bound, and each box's simulated time with the oracle's sum of 2 dt.
Bounds (as in test_gpu_parity.py): FP64 1e-12 of each field family's
largest magnitude; FP32 1e-5 per step on the same float-rounded input.

The benchmark ensemble (64 boxes of {32..256}^3, per-box Mach in [0.5, 3]
and beta in [0.1, 10]) runs 100 graph-replayed steps; every box either
completes them or carries a record, and sampled boxes equal single-grid
handles stepped the same way (which the parity tests pin to the oracle
step by step).
"""
import sys
import time

import numpy as np
import pytest

import oracle
from gpu_util import family_rel_err, max_family_err
from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

NSTEPS = 3
TOL = {"f64": 1e-12, "f32": NSTEPS * 1e-5}
DT_RTOL = {"f64": 1e-14, "f32": 1e-6}


@pytest.fixture(scope="module")
def M():
    from paper_1004_1680_amd import mhd
    mhd.load()
    return mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def uneven_boxes():
    """four smooth boxes of different shapes and a Mach-2 turbulent cube"""
    dims = [(16, 16, 16), (24, 16, 32), (32, 32, 32), (48, 48, 48), (32, 32, 32)]
    ss = [I.random_smooth(n, seed=60 + i) for i, n in enumerate(dims[:4])]
    ss.append(I.turbulence(dims[4], seed=64, mach=2.0, beta=1.0))
    return dims, ss


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ensemble_boxes_match_the_oracle(M, prec):
    say(f"case: ensemble vs oracle, {prec}, {NSTEPS} graph-replayed steps")
    dims, ss = uneven_boxes()
    if prec == "f32":
        ss = [s.astype(np.float32).astype(np.float64) for s in ss]
    B = M.Batch(dims, prec=prec)
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(NSTEPS, graph=True)
    steps, nonphys = B.status()
    assert list(steps) == [NSTEPS] * len(dims) and not nonphys.any()
    times = B.times()
    for i, (n, s) in enumerate(zip(dims, ss)):
        o, t, dts = oracle.run(s, NSTEPS)
        g = B.get_state(i)
        err = family_rel_err(g, o)
        say("box", i, n, "err", {k: f"{v:.2e}" for k, v in err.items()}, "time", times[i], t)
        assert max(err.values()) <= TOL[prec], (i, err)
        assert abs(times[i] - t) <= DT_RTOL[prec] * t, (i, times[i], t)
    B.close()


def test_benchmark_ensemble_hundred_steps(M):
    """64 boxes of {32..256}^3 (seed 4), FP32, 100 steps replayed from one
    captured graph: per-box steps and records, aggregate throughput, and the
    smallest, the largest and a middle box against single-grid handles
    stepped the same 100 times (device dt; bit for bit)"""
    say("case: benchmark ensemble, 100 steps")
    spec = I.ensemble_spec(nbox=64, seed=4)
    dims = [(n, n, n) for n, _, _, _ in spec]
    sizes = [n for n, _, _, _ in spec]
    picks = {sizes.index(min(sizes)), sizes.index(max(sizes)), len(spec) // 2}
    B = M.Batch(dims, prec="f32")
    keep = {}
    for i, (n, m, b, sd) in enumerate(spec):
        s = I.turbulence((n, n, n), seed=sd, mach=m, beta=b)
        B.set_state(i, s)
        if i in picks:
            keep[i] = s
    say("boxes resident; cells", B.ncell)
    B.run(1, graph=True)            # the first (eager) step and the capture
    B.status(raise_on_nonphysical=False)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.run(99, graph=True)
    steps, nonphys = B.status(raise_on_nonphysical=False)
    el = time.perf_counter() - t0
    done = int((steps == 100).sum())
    say(f"100 steps: {done} of 64 boxes completed them, records {sorted(set(nonphys.tolist()))}, "
        f"{int((nonphys != 0).sum())} boxes stopped; 99 replayed steps "
        f"{B.ncell * 99 / el / 1e6:.0f} Mcell-updates/s")
    # a box either completed the run or carries the record that stopped it
    assert all((steps[i] == 100) == (nonphys[i] == 0) for i in range(64))
    for i, s in keep.items():
        S = M.Solver(dims[i], prec="f32")
        S.set_state(s)
        k = 0
        for _ in range(100):
            S.step_auto(0.7)
            try:
                k = S.status()
            except M.NonPhysicalState:
                break
        say("box", i, dims[i], "batch steps", int(steps[i]), "single steps", k, "record", int(nonphys[i]))
        assert k == steps[i]
        assert np.array_equal(B.get_state(i), S.get_state()), i
        S.close()
    B.close()


def test_zero_speed_record_in_an_ensemble(M):
    """a static, cold, unmagnetised box (rho = 1, m = e = b = 0: physical,
    p = 0, but without any signal speed) keeps record 2 (zero signal speed)
    through graph-replayed steps whose CFL the previous step's last launch
    found; its neighbour box advances normally"""
    say("case: zero-speed record in an ensemble")
    n = (16, 16, 16)
    cold = np.zeros((8,) + n)
    cold[0] = 1.0
    other = I.random_smooth((8, 8, 8), seed=3)
    B = M.Batch([n, (8, 8, 8)], prec="f32")
    B.set_state(0, cold)
    B.set_state(1, other)
    B.run(3, graph=True)
    steps, nonphys = B.status(raise_on_nonphysical=False)
    assert list(nonphys) == [2, 0] and list(steps) == [0, 3]
    assert np.array_equal(B.get_state(0), cold)
    o, _, _ = oracle.run(other.astype(np.float32).astype(np.float64), 3)
    assert max_family_err(B.get_state(1), o) <= 3e-5
    B.close()
