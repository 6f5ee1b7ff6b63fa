"""Slope limiter variants (minmod, MC, superbee; the paper's is van Leer's)
on the GPU against the oracle run with the same limiter: every operator
along every axis and full steps, in both tiers, with the tolerances of
test_gpu_parity.py; device-dt steps; switching back to van Leer's restores
the fused path bit for bit; the fused reverse pairs with each variant equal
the two operators bit for bit; argument checks."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import max_family_err
from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
KINDS = [1, 2, 3]          # minmod, MC, superbee


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
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("op", ["fluid", "magnetic"])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_limiter_operator_parity(M, prec, kind, op, d):
    n = (40, 24, 16)
    say(f"case: limiter {kind} {op} d={d} {prec}")
    s = I.random_smooth(n, seed=60 + d)
    if prec == "f32":
        s = f32_round(s)
    dt, c = 0.35 / n[0] / 2.5, 3.1
    S = M.Solver(n, prec=prec)
    S.set_limiter(kind)
    assert S.limiter() == kind
    S.set_state(s)
    S.set_relaxation_speed(c)
    getattr(S, op)(d, dt)
    g = S.get_state()
    S.close()
    if op == "fluid":
        o = oracle.fluid_sweep(s, d, dt, c, limiter=kind)
        ref = oracle.fluid_sweep(s, d, dt, c)
    else:
        o = oracle.mag_sweep(s, d, dt, limiter=kind)
        ref = oracle.mag_sweep(s, d, dt)
    err = max_family_err(g, o)
    say("err", err, "van Leer differs by", max_family_err(o, ref))
    assert err <= TOL[prec]
    # the limiter reached the kernels: the result is the variant's
    assert max_family_err(g, ref) > 10 * err


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", KINDS)
def test_limiter_steps_parity(M, prec, kind):
    n = (32, 24, 16)
    say(f"case: limiter {kind} 3 steps {prec}")
    s = I.random_smooth(n, seed=23)
    if prec == "f32":
        s = f32_round(s)
    S = M.Solver(n, prec=prec)
    S.set_limiter(kind)
    S.set_state(s)
    gdts = S.run(3)
    g = S.get_state()
    S.close()
    o, _, odts = oracle.run(s, 3, limiter=kind)
    assert np.allclose(gdts, odts, rtol=1e-6 if prec == "f32" else 1e-14, atol=0)
    err = max_family_err(g, o)
    say("err", err)
    assert err <= TOL[prec] * (3 if prec == "f32" else 1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("d", [0, 1, 2])
def test_limiter_fused_pair_is_the_two_operators(M, prec, kind, d):
    """the fused reverse pair M_d F_d with a variant limiter equals the two
    operators bit for bit, and the oracle's M_d then F_d"""
    n = (40, 24, 16)
    say(f"case: limiter {kind} fused pair d={d} {prec}")
    s = I.random_smooth(n, seed=31 + d)
    if prec == "f32":
        s = f32_round(s)
    dt, c = 0.35 / n[0] / 2.5, 3.1
    outs = []
    for mode in (1, 2):
        S = M.Solver(n, prec=prec)
        S.set_reverse(mode)
        S.set_limiter(kind)
        S.set_state(s)
        S.set_relaxation_speed(c)
        S.sweep(3 + d, dt)
        outs.append(S.get_state())
        S.close()
    assert np.array_equal(outs[0], outs[1])
    o = oracle.fluid_sweep(oracle.mag_sweep(s, d, dt, limiter=kind), d, dt, c, limiter=kind)
    err = max_family_err(outs[0], o)
    say("err", err)
    assert err <= (2e-5 if prec == "f32" else 1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_limiter_device_steps_and_switch_back(M, prec):
    """device-dt steps with a variant are the same with fused and with
    separate reverse pairs; back on van Leer's, the steps equal a fresh
    handle's from the same state"""
    n = (32, 32, 32)
    say(f"case: limiter device steps, switch back {prec}")
    s = I.random_smooth(n, seed=12)
    out = []
    for reverse in (1, 2):
        S = M.Solver(n, prec=prec)
        S.set_reverse(reverse)
        S.set_limiter(M.MHD_LIMITER_MC)
        S.set_state(s)
        for _ in range(3):
            S.step_auto(0.7)
        assert S.status() == 3
        out.append(S.get_state())
        if reverse == 1:
            mid = out[-1]
            S.set_limiter(M.MHD_LIMITER_VANLEER)
            for _ in range(2):
                S.step_auto(0.7)
            S.status()
            back = S.get_state()
        S.close()
    assert np.array_equal(out[0], out[1])
    R = M.Solver(n, prec=prec)
    R.set_state(mid)
    for _ in range(2):
        R.step_auto(0.7)
    R.status()
    assert np.array_equal(R.get_state(), back)
    R.close()


def test_limiter_key_checks(M):
    S = M.Solver((16, 16, 16), prec="f32")
    assert S.limiter() == M.MHD_LIMITER_VANLEER
    for bad in (-1, 4):
        with pytest.raises(M.MHDError):
            S.set_limiter(bad)
    assert S.limiter() == M.MHD_LIMITER_VANLEER
    S.set_limiter(M.MHD_LIMITER_SUPERBEE)
    assert S.limiter() == M.MHD_LIMITER_SUPERBEE
    # the built-in reverse-pair choice follows the limiter (FP32: fused for
    # van Leer's and minmod, the two operators for MC and superbee); an
    # explicit choice stays
    for kind, want in ((0, 1), (1, 1), (2, 2), (3, 2)):
        S.set_limiter(kind)
        assert S.reverse() == want, kind
    S.set_reverse(1)
    S.set_limiter(M.MHD_LIMITER_SUPERBEE)
    assert S.reverse() == 1
    S.close()


BDIMS = [(16, 16, 16), (24, 16, 32), (8, 12, 16)]


def single_box_steps(M, n, s, kinds_steps):
    S = M.Solver(n, prec="f32")
    S.set_state(s)
    total = 0
    for kind, k in kinds_steps:
        S.set_limiter(kind)
        for _ in range(k):
            S.step_auto(0.7)
        total += k
    assert S.status() == total
    out = S.get_state()
    S.close()
    return out


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("graph", [False, True])
def test_batch_limiter_equals_single_boxes(M, kind, graph):
    """an ensemble with a variant limiter evolves every box bit for bit as
    a single-grid handle with that limiter, eagerly or from a graph"""
    say(f"case: batch limiter {kind} graph={graph}")
    ss = [I.random_smooth(n, seed=70 + i) for i, n in enumerate(BDIMS)]
    ref = [single_box_steps(M, n, s, [(kind, 3)]) for n, s in zip(BDIMS, ss)]
    B = M.Batch(BDIMS, prec="f32")
    B.set_limiter(kind)
    assert B.limiter() == kind
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(3, graph=graph)
    steps, nonphys = B.status()
    assert list(steps) == [3] * len(BDIMS) and not nonphys.any()
    for i in range(len(BDIMS)):
        assert np.array_equal(B.get_state(i), ref[i]), i
    B.close()


def test_batch_limiter_change_recaptures_the_graph(M):
    """graph steps with van Leer's, then with MC: the captured step of the
    first limiter is not replayed for the second"""
    say("case: batch limiter change between graph runs")
    ss = [I.random_smooth(n, seed=80 + i) for i, n in enumerate(BDIMS)]
    ref = [single_box_steps(M, n, s, [(0, 2), (2, 2)]) for n, s in zip(BDIMS, ss)]
    B = M.Batch(BDIMS, prec="f32")
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(2, graph=True)
    B.set_limiter(M.MHD_LIMITER_MC)
    B.run(2, graph=True)
    steps, nonphys = B.status()
    assert list(steps) == [4] * len(BDIMS) and not nonphys.any()
    for i in range(len(BDIMS)):
        assert np.array_equal(B.get_state(i), ref[i]), i
    with pytest.raises(M.MHDError):
        B.set_limiter(5)
    assert B.limiter() == M.MHD_LIMITER_MC
    B.close()
