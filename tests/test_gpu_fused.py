"""The reverse-half pair M_d then F_d of a step in one launch (the fused
kernels; section II.B's symmetric sweep order).

The fused kernels evaluate the same device functions in the same order as
the two operators run one after the other, so they are compared with them
bit for bit: on every axis, on ragged grids (pencils down to the minimum
length 8, shorter than the fused march's 13-cell warm-up), with several
march chunkings, in both tiers, through full steps with the fused CFL, and
on the skip path of a non-physical state.  The pair is also checked against
the oracle's M_d followed by F_d, with the operator tolerances of
test_gpu_parity.py (FP32: twice the one-operator bound for two operators).
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import max_family_err, smooth_state
from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}
FUSED, SEPARATE = 1, 2


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


def solver(M, n, prec, mode, chunk=0):
    S = M.Solver(n, prec=prec)
    S.set_reverse(mode)
    assert S.reverse() == mode
    if chunk:
        for ax in (1, 2):
            if n[ax] % chunk == 0:
                S.set_chunk(ax, chunk)
                S.set_pair_chunk(ax, chunk)
                assert S.pair_chunk(ax) == chunk
    return S


def reverse_pair(M, s, n, prec, d, dt, c, mode, chunk=0):
    S = solver(M, n, prec, mode, chunk)
    S.set_state(s)
    S.set_relaxation_speed(c)
    S.sweep(3 + d, dt)
    out = S.get_state()
    S.close()
    return out


GRIDS = [(40, 24, 16), (16, 48, 20), (8, 8, 8), (12, 8, 36), (512, 8, 12)]   # the last: 512-cell x rows on a thin box


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("d", [0, 1, 2])
def test_fused_pair_is_the_two_operators(M, prec, n, d):
    say(f"case: fused M_{d} F_{d} n={n} {prec}")
    s = smooth_state(n, seed=31 + d)
    if prec == "f32":
        s = f32_round(s)
    dt, c = 0.35 / n[0] / 2.5, 3.1
    fused = reverse_pair(M, s, n, prec, d, dt, c, FUSED)
    separate = reverse_pair(M, s, n, prec, d, dt, c, SEPARATE)
    assert np.array_equal(fused, separate)
    o = oracle.fluid_sweep(oracle.mag_sweep(s, d, dt), d, dt, c)
    err = max_family_err(fused, o)
    say("err vs oracle", err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_pair_chunking(M, prec):
    """the fused march with every chunk length (the warm-up is longer than
    the shortest chunk) gives the separate operators' result"""
    n = (24, 32, 48)
    say(f"case: fused pair chunking {n} {prec}")
    s = I.random_smooth(n, seed=9)
    dt, c = 0.35 / n[0] / 2.5, 3.1
    for d in (1, 2):
        ref = reverse_pair(M, s, n, prec, d, dt, c, SEPARATE)
        for ch in (0, 8, 16):
            out = reverse_pair(M, s, n, prec, d, dt, c, FUSED, ch)
            assert np.array_equal(out, ref), (d, ch)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [(40, 24, 16), (32, 32, 32), (8, 16, 8)])
def test_fused_steps_are_the_separate_steps(M, prec, n):
    """full steps with the device CFL (the fused CFL then rides on the fused
    x pair): states, time steps and times equal the 12-launch steps"""
    say(f"case: fused steps {n} {prec}")
    s = I.random_smooth(n, seed=12)
    res = []
    for mode in (FUSED, SEPARATE):
        S = solver(M, n, prec, mode)
        S.set_state(s)
        for _ in range(4):
            S.step_auto(0.7)
        assert S.status() == 4
        res.append((S.get_state(), S.time()))
        S.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_steps_match_the_oracle(M, prec):
    n = (40, 24, 16)
    say(f"case: fused steps vs oracle {n} {prec}")
    s = I.random_smooth(n, seed=23)
    if prec == "f32":
        s = f32_round(s)
    S = solver(M, n, prec, FUSED)
    S.set_state(s)
    dts = S.run(3)
    g = S.get_state()
    S.close()
    o, _, odts = oracle.run(s, 3)
    assert np.allclose(dts, odts, rtol=1e-6 if prec == "f32" else 1e-14)
    err = max_family_err(g, o)
    say("err", err)
    assert err <= (3e-5 if prec == "f32" else 1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_pair_keeps_a_nonphysical_state(M, prec):
    """after a non-physical state is recorded the fused kernels copy every
    field unchanged, like the separate operators"""
    n = (32, 32, 32)
    say(f"case: fused pair skip path {prec}")
    s = I.random_smooth(n, seed=6)
    bad = s.copy()
    bad[4, 3, 5, 7] = -1.0          # negative energy: p < 0
    S = solver(M, n, prec, FUSED)
    S.set_state(bad)
    before = S.get_state()
    for _ in range(2):
        S.step_auto(0.7)
    with pytest.raises(M.NonPhysicalState):
        S.status()
    assert np.array_equal(S.get_state(), before)
    S.close()


def test_reverse_key_checks(M):
    S = M.Solver((16, 16, 16), prec="f32")
    assert S.reverse() == FUSED
    S.set_reverse(SEPARATE)
    assert S.reverse() == SEPARATE
    S.set_reverse(0)
    assert S.reverse() == FUSED
    with pytest.raises(M.MHDError):
        S.set_reverse(3)
    # the pair chunks are separate launch keys with the chunk rules
    S.set_chunk(1, 8)
    S.set_pair_chunk(1, 16)
    assert (S.chunk(1), S.pair_chunk(1)) == (8, 16)
    S.set_pair_chunk(1, 0)
    assert S.chunk(1) == 8 and S.pair_chunk(1) in (8, 16)
    with pytest.raises(M.MHDError):
        S.set_pair_chunk(2, 12)
    S.close()
    S = M.Solver((16, 16, 16), prec="f64")
    assert S.reverse() == SEPARATE
    S.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", [FUSED, SEPARATE])
def test_wide_offsets_give_the_same_steps(M, prec, mode):
    """the y and z sweeps address memory with 32-bit byte offsets where every
    offset fits (all grids here) and with 64-bit arithmetic otherwise (fields
    over 4 GiB); forcing the second path gives the same steps bit for bit"""
    n = (32, 24, 40)
    say(f"case: wide offsets {prec} reverse={mode}")
    s = I.random_smooth(n, seed=8)
    outs = []
    for wide in (0, 1):
        S = solver(M, n, prec, mode, chunk=8)
        S.set_launch(M.MHD_TUNE_WIDE_OFFSETS, wide)
        assert S.launch(M.MHD_TUNE_WIDE_OFFSETS) == wide
        S.set_state(s)
        for _ in range(3):
            S.step_auto(0.7)
        S.status()
        outs.append(S.get_state())
        S.close()
    assert np.array_equal(outs[0], outs[1])


def test_batch_wide_offsets_give_the_same_steps(M):
    dims = [(16, 16, 16), (24, 16, 32), (8, 12, 16)]
    say("case: batch wide offsets")
    ss = [I.random_smooth(n, seed=50 + i) for i, n in enumerate(dims)]
    outs = []
    for wide in (0, 1):
        B = M.Batch(dims, prec="f32")
        B.set_launch(M.MHD_BATCH_WIDE_OFFSETS, wide)
        assert B.launch(M.MHD_BATCH_WIDE_OFFSETS) == wide
        for i, st in enumerate(ss):
            B.set_state(i, st)
        B.run(2, graph=True)
        B.status()
        outs.append([B.get_state(i) for i in range(len(dims))])
        B.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", [FUSED, SEPARATE])
def test_sweep_with_fused_cfl(M, prec, mode):
    """sweep code 6 (the reverse x pair that also finds the CFL maximum of
    its result, the last launch of a step) followed by device-dt steps equals
    sweep code 3 followed by the same steps, whose first CFL is then a
    separate reduction"""
    n = (32, 24, 16)
    say(f"case: sweep 6 {prec} reverse={mode}")
    s = I.random_smooth(n, seed=14)
    outs = []
    for code in (6, 3):
        S = solver(M, n, prec, mode)
        S.set_state(s)
        dt = 0.5 * S.cfl_dt(0.7)
        S.sweep(code, dt)
        for _ in range(2):
            S.step_auto(0.7)
        assert S.status() == 2
        outs.append((S.get_state(), S.time()))
        S.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zero_speed_record_survives_the_fused_cfl(M, prec):
    """a static, cold, unmagnetised state (rho = 1, m = e = b = 0) is
    physical (p = 0) but has no signal speed: the device CFL records a zero
    speed (MHD_EINVAL from status, not MHD_ENONPHYS), the steps keep the
    state, and the record stays the same through the CFL that the skipped
    last launch of a step hands to the next step"""
    n = (16, 16, 16)
    say(f"case: zero-speed record {prec}")
    cold = np.zeros((8,) + n)
    cold[0] = 1.0
    S = M.Solver(n, prec=prec)
    S.set_state(cold)
    for rounds in range(2):
        for _ in range(3):
            S.step_auto(0.7)
        with pytest.raises(M.MHDError) as e:
            S.status()
        assert not isinstance(e.value, M.NonPhysicalState), rounds
        assert e.value.code == M.MHD_EINVAL, rounds
    assert np.array_equal(S.get_state(), cold)
    S.close()
