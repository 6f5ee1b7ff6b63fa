"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances:
 * FP64 tier: 1e-12 relative to the largest magnitude of each field family
   (rho; m; e; b) -- both sides evaluate the same expressions in the same
   order without fused multiply-adds, so the observed difference is 0 or a
   few ulp;
 * FP32 tier: 1e-5 of the same norm after one step or one operator, against
   the oracle run on the same float-rounded input; 1e-4 relative L1 after
   100 steps of a smooth wave.
Results that do not depend on rounding (uniform states, axis symmetry,
chunking, determinism, checkpointing) are compared bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import family_rel_err, l1_rel, max_family_err, smooth_state
from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


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


def rotate(s):
    t = np.transpose(s, (0, 2, 3, 1))
    return t[[0, 3, 1, 2, 4, 7, 5, 6]].copy()


def gpu_run(M, s, n, prec, nsteps, cfl=0.7):
    S = M.Solver(n, prec=prec)
    S.set_state(s)
    dts = S.run(nsteps, cfl)
    out = S.get_state()
    t = S.time()
    S.close()
    return out, dts, t


# ---------------------------------------------------------------------------
# the 32^3 FP64 fast-wave case: 10 steps, field by field
# ---------------------------------------------------------------------------

def test_c1_fast_wave_fp64_ten_steps(M):
    n = (32, 32, 32)
    say("case: 32^3 FP64 fast wave, 10 steps")
    s0 = I.linear_wave(n, "fast", 1e-6, (1.0, 0.0, 0.0))
    g, gdts, gt = gpu_run(M, s0, n, "f64", 10)
    o, t, odts = oracle.run(s0, 10)
    assert np.allclose(gdts, odts, rtol=1e-14, atol=0)
    assert gt == pytest.approx(t, rel=1e-14)
    err = family_rel_err(g, o)
    say("family errors", err)
    assert max(err.values()) <= TOL["f64"], err


# ---------------------------------------------------------------------------
# every operator along every axis, on ragged grids
# ---------------------------------------------------------------------------

GRIDS = [(40, 24, 16), (16, 48, 20), (8, 8, 8), (512, 8, 12)]   # the last: 512-cell x rows on a thin box


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("op", ["fluid", "magnetic"])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_operator_parity(M, prec, n, op, d):
    say(f"case: {op} d={d} n={n} {prec}")
    s = smooth_state(n, seed=17 + d)
    if prec == "f32":
        s = f32_round(s)
    dt, c = 0.35 / n[0] / 2.5, 3.1
    S = M.Solver(n, prec=prec)
    S.set_state(s)
    S.set_relaxation_speed(c)
    getattr(S, op)(d, dt)
    g = S.get_state()
    o = oracle.fluid_sweep(s, d, dt, c) if op == "fluid" else oracle.mag_sweep(s, d, dt)
    err = max_family_err(g, o)
    say("err", err)
    assert err <= TOL[prec]
    # the operator leaves the other family bit-identical
    keep = slice(5, 8) if op == "fluid" else slice(0, 5)
    assert np.array_equal(g[keep], s[keep])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_brio_wu_shock_tube_parity(M, prec, axis):
    """a discontinuous state along each axis (gamma = 2): both limiters clip
    at the jumps and the CT chains cross the jump of b_t; FP64 over 10 steps,
    FP32 over one step, against the oracle"""
    n = [8, 8, 8]
    n[axis] = 64
    n = tuple(n)
    say(f"case: Brio-Wu tube along {'xyz'[axis]} {n} {prec}")
    s = I.brio_wu(n, axis)
    steps = 10 if prec == "f64" else 1
    if prec == "f32":
        s = f32_round(s)
    S = M.Solver(n, gamma=2.0, prec=prec)
    S.set_state(s)
    gdts = S.run(steps)
    g = S.get_state()
    S.close()
    o, _, odts = oracle.run(s, steps, gamma=2.0)
    assert np.allclose(gdts, odts, rtol=1e-14 if prec == "f64" else 1e-6, atol=0)
    err = max_family_err(g, o)
    say("err", err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_field_loop_parity(M, prec):
    """the advected field loop (weak b, jump of b at the loop's edge, b_z = 0):
    FP64 over 20 steps, FP32 over one step, against the oracle"""
    n = (64, 32, 8)
    say(f"case: field loop {n} {prec}")
    s = I.field_loop(n)
    steps = 20 if prec == "f64" else 1
    if prec == "f32":
        s = f32_round(s)
    g, gdts, _ = gpu_run(M, s, n, prec, steps)
    o, _, odts = oracle.run(s, steps)
    assert np.allclose(gdts, odts, rtol=1e-14 if prec == "f64" else 1e-6, atol=0)
    err = max_family_err(g, o)
    say("err", err)
    assert err <= TOL[prec]
    assert np.abs(g[7]).max() == 0.0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_chunked_march_is_bitwise_equal(M, prec):
    n = (24, 32, 48)
    say(f"case: chunked march {n} {prec}")
    s = I.random_smooth(n, seed=5)
    outs = []
    for ch in (0, 8, 16):
        S = M.Solver(n, prec=prec)
        if ch:
            S.set_chunk(1, ch)
            S.set_chunk(2, ch)
        S.set_state(s)
        S.run(2)
        outs.append(S.get_state())
        S.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [(40, 24, 16), (32, 32, 32)])
def test_full_step_parity(M, prec, n):
    say(f"case: 3 full steps {n} {prec}")
    s = I.random_smooth(n, seed=23)
    if prec == "f32":
        s = f32_round(s)
    g, gdts, _ = gpu_run(M, s, n, prec, 3)
    o, _, odts = oracle.run(s, 3)
    assert np.allclose(gdts, odts, rtol=1e-6 if prec == "f32" else 1e-14)
    err = max_family_err(g, o)
    say("err", err)
    assert err <= TOL[prec] * (3 if prec == "f32" else 1)


# ---------------------------------------------------------------------------
# exact properties on the GPU
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_uniform_state_bit_identical(M, prec):
    n = (16, 12, 8)
    say(f"case: uniform {prec}")
    s = f32_round(I.uniform(n, rho=1.3, v=(0.3, -0.7, 0.2), p=0.9, b=(0.4, -1.1, 0.6)))
    g, _, _ = gpu_run(M, s, n, prec, 3)
    assert np.array_equal(g, s)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("op", ["fluid", "magnetic"])
def test_cyclic_axis_symmetry_bitwise(M, prec, op):
    # the x (row) kernels and the y, z (march) kernels evaluate the same
    # expressions: a relabelled state swept along d+1 equals the relabelled
    # result of the sweep along d, bit for bit
    s = f32_round(I.random_smooth((16, 8, 32), seed=5))
    tau, c = 0.25, 3.0
    say(f"case: cyclic symmetry {op} {prec}")
    for d in range(3):
        r = rotate(s)
        outs = []
        for state, dd in ((s, d), (r, (d + 1) % 3)):
            n = (state.shape[3], state.shape[2], state.shape[1])
            S = M.Solver(n, prec=prec)
            S.set_state(state)
            S.set_relaxation_speed(c)
            getattr(S, op)(dd, tau / n[0])
            outs.append(S.get_state())
            S.close()
        assert np.array_equal(rotate(outs[0]), outs[1]), (op, d)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_conservation_and_div_b(M, prec):
    n = (32, 24, 16)
    say(f"case: conservation {prec}")
    # FP32 rounding of a div-free field leaves div b at the FP32 roundoff
    # level; the FP64 tier starts exactly div-free
    s = I.random_smooth(n, seed=3, amp_b=0.25)
    if prec == "f32":
        s = f32_round(s)
    S = M.Solver(n, prec=prec)
    S.set_state(s)
    d0 = S.diag()
    S.run(5)
    d1 = S.diag()
    scale = np.array([np.abs(s[f]).mean() for f in range(8)]) * (n[1] / n[0]) * (n[2] / n[0])
    eps = 1e-13 if prec == "f64" else 2e-6
    assert np.all(np.abs(d1[:8] - d0[:8]) <= eps * scale + 1e-300), (d0, d1)
    if prec == "f64":
        assert d0[8] < 1e-14 and d1[8] < 1e-13, (d0[8], d1[8])
    else:
        assert d1[8] <= d0[8] + 1e-6, (d0[8], d1[8])


def test_cfl_parity_and_relaxation_speed(M):
    n = (40, 24, 16)
    s = I.random_smooth(n, seed=9)
    for prec in ("f64", "f32"):
        say(f"case: cfl {prec}")
        si = s if prec == "f64" else f32_round(s)
        S = M.Solver(n, prec=prec)
        S.set_state(si)
        with pytest.raises(M.MHDError):
            S.step(1e-3)          # relaxation speed not set yet
        dt = S.cfl_dt(0.7)
        odt, ovmax = oracle.cfl(si, 0.7)
        assert dt == pytest.approx(odt, rel=1e-15)
        assert S.relaxation_speed() == pytest.approx(ovmax, rel=1e-15)


@pytest.mark.parametrize("plant", ["negative_pressure", "negative_density", "nan"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cfl_flags_nonphysical(M, plant, prec):
    say(f"case: nonphysical {plant} {prec}")
    s = I.uniform((16, 8, 8))
    if plant == "negative_pressure":
        s[4, 2, 3, 4] = 0.1
    elif plant == "negative_density":
        s[0, 1, 1, 1] = -1.0
    else:
        s[2, 5, 5, 5] = np.nan
    S = M.Solver((16, 8, 8), prec=prec)
    S.set_state(s)
    with pytest.raises(M.NonPhysicalState):
        S.cfl_dt()
    # the device-side path records it and leaves the state unchanged
    S.step_auto(0.7)
    with pytest.raises(M.NonPhysicalState):
        S.status()
    g = S.get_state()
    ref = s if prec == "f64" else f32_round(s)
    assert np.array_equal(np.isnan(g), np.isnan(ref))
    assert np.array_equal(np.nan_to_num(g), np.nan_to_num(ref))


def test_diag_parity(M):
    n = (40, 24, 16)
    s = I.random_smooth(n, seed=4)
    say("case: diag")
    S = M.Solver(n, prec="f64")
    S.set_state(s)
    g = S.diag()
    o = oracle.diag(s)
    assert np.allclose(g[:8], o[:8], rtol=1e-13, atol=1e-15)
    assert abs(g[8] - o[8]) < 1e-15


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_deterministic(M, prec):
    n = (32, 16, 24)
    say(f"case: determinism {prec}")
    s = I.random_smooth(n, seed=12)
    a, _, _ = gpu_run(M, s, n, prec, 3)
    b, _, _ = gpu_run(M, s, n, prec, 3)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_checkpoint_resume_bitwise(M, prec):
    n = (24, 16, 32)
    say(f"case: checkpoint {prec}")
    s = I.random_smooth(n, seed=2)
    full, _, _ = gpu_run(M, s, n, prec, 6)
    half, _, _ = gpu_run(M, s, n, prec, 3)
    rest, _, _ = gpu_run(M, half, n, prec, 3)
    assert np.array_equal(full, rest)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_step_auto_matches_host_path(M, prec):
    n = (32, 24, 16)
    say(f"case: step_auto {prec}")
    s = I.random_smooth(n, seed=8)
    host, dts, t = gpu_run(M, s, n, prec, 4)
    S = M.Solver(n, prec=prec)
    S.set_state(s)
    for _ in range(4):
        S.step_auto(0.7)
    assert S.status() == 4
    assert np.array_equal(S.get_state(), host)
    assert S.time() == t


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_cfl_follows_state_changes(M, prec):
    """step_auto takes the CFL of a step from the previous step's last
    operator while the state is unchanged, and recomputes it after a single
    operator or a new state: every step equals the host path (cfl_dt + step)
    bit for bit"""
    n = (32, 32, 32)
    say(f"case: fused CFL and state changes {prec}")
    s1 = I.random_smooth(n, seed=4)
    s2 = I.random_smooth(n, seed=5)
    A = M.Solver(n, prec=prec)
    B = M.Solver(n, prec=prec)
    A.set_state(s1)
    B.set_state(s1)
    for _ in range(3):
        A.step_auto(0.7)
        dtb = B.cfl_dt(0.7)
        B.step(dtb)
    # a single operator (both with the relaxation speed of the last CFL):
    # the fused CFL of A is stale afterwards
    dt = 0.3 * dtb
    A.fluid(1, dt)
    B.fluid(1, dt)
    for _ in range(2):
        A.step_auto(0.7)
        B.step(B.cfl_dt(0.7))
    assert np.array_equal(A.get_state(), B.get_state())
    A.set_state(s2)
    B.set_state(s2)
    for _ in range(3):
        A.step_auto(0.7)
        B.step(B.cfl_dt(0.7))
    A.status()
    assert np.array_equal(A.get_state(), B.get_state())
    assert A.time() == B.time()


SCREEN_STATES = {
    # every cell ties for the largest signal speed
    "uniform": lambda n: I.uniform(n, rho=1.3, v=(0.4, -0.7, 0.2), p=0.8, b=(0.5, 0.3, -0.2)),
    # p about 1e-7 of e: the FP32 screen is never sure, every cell takes FP64
    "cold": lambda n: I.uniform(n, rho=1.0, v=(1.0, 0.5, 0.0), p=1e-7, b=(0.0, 0.0, 0.0)),
    # shorter waves and larger amplitudes than the default smooth state
    "rough": lambda n: I.random_smooth(n, seed=21, amp_v=0.25, amp_b=0.2, kmax=2),
}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", sorted(SCREEN_STATES))
def test_fused_cfl_screen_is_exact(M, prec, kind):
    """the fused CFL of the FP32 tier evaluates in FP64 only the cells that
    may raise the running maximum or may be non-physical; the maximum and
    the steps stay those of the full FP64 reduction, bit for bit"""
    n = (32, 24, 16)
    say(f"case: fused CFL screen {kind} {prec}")
    s = SCREEN_STATES[kind](n)
    A = M.Solver(n, prec=prec)
    B = M.Solver(n, prec=prec)
    A.set_state(s)
    B.set_state(s)
    for _ in range(4):
        A.step_auto(0.7)
        B.step(B.cfl_dt(0.7))
    assert A.status() == 4
    assert np.array_equal(A.get_state(), B.get_state())
    assert A.time() == B.time()
    A.close()
    B.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_cfl_carries_a_nonphysical_record(M, prec):
    """a non-physical state stops every step; the record survives the
    fused-CFL hand-over between steps, and a new state clears the path"""
    n = (32, 32, 32)
    say(f"case: fused CFL non-physical record {prec}")
    s = I.random_smooth(n, seed=6)
    bad = s.copy()
    bad[4, 3, 5, 7] = -1.0          # negative energy: p < 0
    S = M.Solver(n, prec=prec)
    S.set_state(bad)
    before = S.get_state()
    for _ in range(3):
        S.step_auto(0.7)
    with pytest.raises(M.NonPhysicalState):
        S.status()
    assert np.array_equal(S.get_state(), before)
    S.set_state(s)
    host, _, _ = gpu_run(M, s, n, prec, 2)
    for _ in range(2):
        S.step_auto(0.7)
    assert S.status() == 2
    assert np.array_equal(S.get_state(), host)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("r", [2, 3, 4, 8])
def test_restriction_parity(M, prec, r):
    # r = 2, 4, 8: the fixed-factor kernel; r = 3: the general one
    say(f"case: restrict by {r} {prec}")
    nf = (16 * r, 8 * r, 8 * r)
    s = I.random_smooth(nf, seed=6)
    if prec == "f32":
        s = f32_round(s)
    F = M.Solver(nf, prec=prec)
    F.set_state(s)
    C = M.Solver((nf[0] // r, nf[1] // r, nf[2] // r), prec=prec)
    F.restrict_to(C)
    g = C.get_state()
    o = oracle.restrict(s, r)
    assert max_family_err(g, o) <= (1e-15 if prec == "f64" else 1e-7)
    # totals kept (b totals too, since the fine b is div-free up to the
    # rounding of the input) and the coarse div b is the block mean of the
    # fine one
    dc, df = C.diag(), F.diag()
    scale = np.array([np.abs(s[f]).mean() for f in range(8)]) * 0.25
    eps = 1e-13 if prec == "f64" else 1e-6
    assert np.all(np.abs(dc[:8] - df[:8]) <= eps * scale), (dc, df)
    assert dc[8] < (1e-13 if prec == "f64" else 1e-6)


def test_restriction_rejects_mismatched_grids(M):
    F = M.Solver((64, 32, 32), prec="f32")
    C = M.Solver((16, 16, 8), prec="f32")
    with pytest.raises(M.MHDError):
        F.restrict_to(C)
    C2 = M.Solver((16, 8, 8), prec="f64")
    with pytest.raises(M.MHDError):
        F.restrict_to(C2)


def test_invalid_arguments(M):
    S = M.Solver((16, 8, 8), prec="f32")
    S.set_state(I.uniform((16, 8, 8)))
    S.cfl_dt()
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(M.MHDError):
            S.step(bad)
    with pytest.raises(M.MHDError):
        S.sweep(8, 0.01)
    with pytest.raises(M.MHDError):
        S.fluid(3, 0.01)
    with pytest.raises(M.MHDError):
        S.set_chunk(1, 3)
    with pytest.raises(ValueError):
        S.set_state(np.zeros((8, 8, 8, 8)))


# ---------------------------------------------------------------------------
# precision tiers on the benchmark-family inputs
# ---------------------------------------------------------------------------

def test_turbulence_256_one_step_fp32_and_fp64(M):
    # 256^3 random-phase solenoidal turbulence, rms Mach 1, beta 1 (seed 2)
    n = (256, 256, 256)
    say("case: 256^3 turbulence, 1 step, oracle + FP64 + FP32")
    s = I.turbulence(n, seed=2)
    o, _, _ = oracle.run(s, 1)
    g64, _, _ = gpu_run(M, s, n, "f64", 1)
    e64 = max_family_err(g64, o)
    say("fp64 err", e64)
    assert e64 <= TOL["f64"]
    del g64
    g32, _, _ = gpu_run(M, s, n, "f32", 1)
    e32 = family_rel_err(g32, o)
    say("fp32 err", e32)
    assert max(e32.values()) <= TOL["f32"]


@pytest.mark.parametrize("wave", ["cpaw", "fast"])
def test_fp32_smooth_wave_100_steps(M, wave):
    n = (64, 64, 64)
    say(f"case: 100 steps FP32 {wave} 64^3")
    if wave == "cpaw":
        s = I.cpaw(n, amp=0.1, p0=0.1)
    else:
        s = I.diagonal_wave(n, "fast", amp=1e-2, B=(1.0, 0.6, 0.4))
    o, _, _ = oracle.run(s, 100)
    g, _, _ = gpu_run(M, s, n, "f32", 100)
    e = l1_rel(g, o)
    say("L1", e)
    assert e <= 1e-4
