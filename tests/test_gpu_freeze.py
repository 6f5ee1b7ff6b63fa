"""Freezing-speed variants of the fluid operator on the GPU against the
oracle run with the same variant (section II.B leaves the relaxation speed
open; the method's reading is one speed per step, the CFL speed): the
per-cell speed |v_n| + c_fast and its per-pencil maximum, each from the
state of each stage.  Every axis on ragged grids (x rows of 40 and 8 cells,
march pencils of 24, 16, 12 and 36), device-dt steps, both tiers, with the
tolerances of test_gpu_parity.py; switching back restores the step's speed
and the fused path bit for bit; argument checks."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import max_family_err
from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
MODES = {"cell": 1, "pencil": 2}


@pytest.fixture(scope="module")
def M():
    from paper_1004_1680_amd import mhd
    mhd.load()
    return mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32_round(s):
    return s.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["cell", "pencil"])
@pytest.mark.parametrize("n", [(40, 24, 16), (8, 12, 36)])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_freeze_fluid_operator_parity(M, prec, mode, n, d):
    fr = MODES[mode]
    say(f"case: freeze {mode} fluid d={d} n={n} {prec}")
    s = I.random_smooth(n, seed=70 + d)
    if prec == "f32":
        s = f32_round(s)
    dt = 0.35 / n[0] / 2.5
    S = M.Solver(n, prec=prec)
    S.set_freezing(fr)
    assert S.freezing() == fr
    S.set_state(s)             # no relaxation speed is needed by the variants
    S.fluid(d, dt)
    g = S.get_state()
    S.close()
    o = oracle.fluid_sweep(s, d, dt, 0.0, freeze=fr)
    ref = oracle.fluid_sweep(s, d, dt, oracle.cfl(s)[1])
    err = max_family_err(g, o)
    say("err", err, "the step's speed differs by", max_family_err(o, ref))
    assert err <= TOL[prec]
    assert max_family_err(g, ref) > 10 * err      # the variant reached the kernel


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["cell", "pencil"])
def test_freeze_steps_parity(M, prec, mode):
    """three device-dt steps (the last launch of a step also finds the next
    CFL) against the oracle's three steps with the same variant"""
    fr = MODES[mode]
    n = (32, 24, 16)
    say(f"case: freeze {mode} 3 steps {prec}")
    s = I.random_smooth(n, seed=24)
    if prec == "f32":
        s = f32_round(s)
    S = M.Solver(n, prec=prec)
    S.set_freezing(fr)
    S.set_state(s)
    for _ in range(3):
        S.step_auto(0.7)
    assert S.status() == 3
    g, t = S.get_state(), S.time()
    S.close()
    o, to, _ = oracle.run(s, 3, freeze=fr)
    err = max_family_err(g, o)
    say("err", err, "time", t, to)
    assert err <= 3 * TOL[prec]
    assert t == pytest.approx(to, rel=1e-6 if prec == "f32" else 1e-14)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_freeze_back_to_the_step_speed(M, prec):
    """setting the step's speed again gives the default kernels' steps (fused
    reverse pairs in FP32) bit for bit"""
    n = (24, 16, 32)
    say(f"case: freeze back to the step's speed {prec}")
    s = I.random_smooth(n, seed=25)
    outs = []
    for modes in ((0,), (2, 0)):
        S = M.Solver(n, prec=prec)
        for m in modes:
            S.set_freezing(m)
        S.set_state(s)
        for _ in range(2):
            S.step_auto(0.7)
        S.status()
        outs.append(S.get_state())
        S.close()
    assert np.array_equal(outs[0], outs[1])


def test_freeze_argument_checks(M):
    S = M.Solver((16, 16, 16), prec="f32")
    assert S.freezing() == 0
    with pytest.raises(M.MHDError):
        S.set_freezing(3)
    S.set_freezing(1)
    assert S.reverse() == 2                  # the reverse pairs run as two launches
    with pytest.raises(M.MHDError):
        S.set_limiter(M.MHD_LIMITER_MINMOD)   # variants come with van Leer's only
    S.set_freezing(0)
    S.set_limiter(M.MHD_LIMITER_MINMOD)
    with pytest.raises(M.MHDError):
        S.set_freezing(2)
    S.close()
