"""Parity of the BF16 MFMA closure kernels with the FP64 closure oracle.

Single layers are compared on exactly the BF16 values the kernels consume
(inputs given in BF16, weights rounded to BF16 on both sides): the only
difference is FP32 vs FP64 accumulation, bound 1e-5 of the output scale.
The whole network rounds its hidden activations to BF16 as well, which the
FP64 oracle does not: 3e-2 relative L2 for the correction and the gradient
(a few BF16 ulps, 2^-8 each, through three layers), and the gradient
direction within cosine 0.999."""
import sys

import numpy as np
import pytest

import bf16
from oracle import closure as C
from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

N3 = (32, 32, 64)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1004_1680_amd import mhd
    mhd.load()
    return torch, mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_bf16(torch, a):
    return torch.from_numpy(bf16.bits(a).view(np.int16)).cuda()


@pytest.mark.parametrize("cin,cout", [(8, 32), (32, 32), (32, 8), (8, 8)])
def test_conv_forward_parity(env, cin, cout):
    torch, mhd = env
    say(f"case: conv forward {cin}->{cout}")
    rng = np.random.default_rng(cin * 7 + cout)
    N = int(np.prod(N3))
    x = bf16.round(rng.normal(size=(N, cin)))
    w = rng.normal(size=(27, cin, cout)) / np.sqrt(27 * cin)
    b = rng.normal(size=cout)
    y = torch.empty((N, cout), dtype=torch.float32, device="cuda")
    mhd.conv3d_forward(N3, dev_bf16(torch, x), w, b, y)
    ref = C.conv3d(x, bf16.round(w), b.astype(np.float32).astype(np.float64), N3)
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    say("err", err)
    assert err < 1e-5


@pytest.mark.parametrize("cin,cout", [(8, 32), (32, 32), (32, 8)])
def test_conv_dgrad_parity(env, cin, cout):
    torch, mhd = env
    say(f"case: conv dgrad {cin}->{cout}")
    rng = np.random.default_rng(cin * 5 + cout)
    N = int(np.prod(N3))
    dy = bf16.round(rng.normal(size=(N, cout)))
    w = rng.normal(size=(27, cin, cout)) / np.sqrt(27 * cout)
    dx = torch.empty((N, cin), dtype=torch.float32, device="cuda")
    mhd.conv3d_dgrad(N3, dev_bf16(torch, dy), w, dx)
    ref = C.conv3d_dgrad(dy, bf16.round(w), N3)
    err = np.abs(dx.cpu().numpy() - ref).max() / np.abs(ref).max()
    say("err", err)
    assert err < 1e-5


@pytest.mark.parametrize("cin,cout", [(8, 32), (32, 32), (32, 8), (8, 8)])
def test_conv_wgrad_parity(env, cin, cout):
    torch, mhd = env
    say(f"case: conv wgrad {cin}->{cout}")
    rng = np.random.default_rng(cin * 3 + cout)
    N = int(np.prod(N3))
    x = bf16.round(rng.normal(size=(N, cin)))
    dy = bf16.round(rng.normal(size=(N, cout)))
    dw, db = mhd.conv3d_wgrad(N3, cin, cout, dev_bf16(torch, x.T.copy()), dev_bf16(torch, dy.T.copy()))
    rdw, rdb = C.conv3d_wgrad(x, dy, N3, cin, cout)
    # FP32 sums of 65536 products of unit-variance values
    assert np.abs(dw - rdw).max() < 1e-5 * np.abs(rdw).max() + 2e-3
    assert np.allclose(db, rdb, rtol=1e-5, atol=1e-3)


def closure_problem(seed=0, n=N3):
    """a smooth coarse state, random parameters and a target correction"""
    rng = np.random.default_rng(seed)
    u = I.random_smooth(n, seed=seed + 5).astype(np.float32).astype(np.float64)
    mean = u.reshape(8, -1).mean(axis=1)
    std = u.reshape(8, -1).std(axis=1) + 1e-3
    ps = C.init_params(seed + 1)
    ps[-2] = ps[-2] * 10.0            # a correction of visible size
    out_scale = rng.uniform(0.5, 1.5, 8) * 1e-3
    target = rng.normal(size=(8, int(np.prod(n)))) * 1e-3
    tscale = np.full(8, 1e-3)
    return u, mean, std, ps, out_scale, target, tscale


def setup_closure(torch, mhd, prob, n=N3):
    u, mean, std, ps, out_scale, target, tscale = prob
    cl = mhd.Closure(n)
    cl.set_params(C.flatten(ps).astype(np.float32))
    cl.set_scales(mean, std, out_scale, tscale)
    return cl


def oracle_inputs(prob):
    u, mean, std, ps, out_scale, target, tscale = prob
    # the same BF16 rounding points the kernels apply to weights and input;
    # biases and scales enter in FP32
    x = bf16.round(C.normalize(u.reshape(8, -1), mean.astype(np.float32), std.astype(np.float32)))
    psr = [bf16.round(p) if p.ndim == 3 else p.astype(np.float32).astype(np.float64) for p in ps]
    return x, psr, out_scale.astype(np.float32).astype(np.float64), target.astype(np.float32), tscale


def test_network_forward_and_gradient_parity(env):
    torch, mhd = env
    say("case: closure network forward + gradient")
    prob = closure_problem()
    u, mean, std, ps, out_scale, target, tscale = prob
    cl = setup_closure(torch, mhd, prob)
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    td = torch.from_numpy(target.astype(np.float32).reshape(u.shape)).cuda()
    delta = cl.forward(ud).cpu().numpy().reshape(8, -1)
    x, psr, osc, tgt, ts = oracle_inputs(prob)
    ref = C.forward(x, psr, osc, N3)
    e_fwd = np.linalg.norm(delta - ref) / np.linalg.norm(ref)
    say("forward rel L2", e_fwd)
    assert e_fwd < 3e-2
    L, g = cl.grad(ud, td)
    Lr, gr = C.loss_and_grad(x, psr, osc, tgt.astype(np.float64), ts, N3)
    gr = C.flatten(gr)
    e_g = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    cos = float(np.dot(g, gr) / np.linalg.norm(g) / np.linalg.norm(gr))
    say("loss", L, Lr, "grad rel L2", e_g, "cos", cos)
    assert L == pytest.approx(Lr, rel=1e-3)
    assert e_g < 3e-2 and cos > 0.999
    # per parameter group: agreement where the exact gradient carries signal;
    # the output bias has an exactly zero gradient (the projection removes
    # any uniform output), where the GPU keeps only BF16 rounding noise
    k = 0
    gnorm = np.linalg.norm(gr)
    for p in C.unflatten(gr):
        seg = g[k:k + p.size]
        k += p.size
        if np.linalg.norm(p) > 1e-6 * gnorm:
            assert np.linalg.norm(seg - p.ravel()) < 5e-2 * np.linalg.norm(p)
        else:
            assert np.linalg.norm(seg) < 1e-3 * gnorm


def test_correction_keeps_totals_and_div_b(env):
    torch, mhd = env
    say("case: closure correction invariants")
    prob = closure_problem(seed=3)
    u = prob[0]
    cl = setup_closure(torch, mhd, prob)
    d = cl.forward(torch.from_numpy(u.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    n = N3
    for f in range(5):
        assert abs(d[f].sum()) < 1e-5 * np.abs(d[f]).sum()
    bx, by, bz = d[5], d[6], d[7]
    div = (np.roll(bx, -1, 2) - bx) + (np.roll(by, -1, 1) - by) + (np.roll(bz, -1, 0) - bz)
    assert np.abs(div).max() < 1e-5 * np.abs(d[5:]).max()


def test_training_reduces_the_loss(env):
    torch, mhd = env
    say("case: closure training")
    prob = closure_problem(seed=4)
    u, target = prob[0], prob[5]
    cl = setup_closure(torch, mhd, prob)
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    td = torch.from_numpy(target.astype(np.float32).reshape(u.shape)).cuda()
    # target: what a fixed "teacher" net would output, so it is learnable
    teacher = mhd.Closure(N3)
    tp = C.flatten(C.init_params(9)).astype(np.float32)
    teacher.set_params(tp)
    teacher.set_scales(prob[1], prob[2], prob[4], prob[6])
    td = teacher.forward(ud)
    losses = [cl.train_step(ud, td, 2e-3) for _ in range(40)]
    say("loss", losses[0], losses[-1])
    assert losses[-1] < 0.3 * losses[0]


def test_closure_step_falls_back_on_unphysical_correction(env):
    torch, mhd = env
    say("case: closure guard")
    n = N3
    s = I.random_smooth(n, seed=8)
    prob = closure_problem(seed=2)
    stream = torch.cuda.current_stream()
    cl = mhd.Closure(n, stream=stream)
    ps = C.init_params(3)
    cl.set_params(C.flatten(ps).astype(np.float32))
    big = np.full(8, 1e3, dtype=np.float32)     # absurd correction
    cl.set_scales(prob[1], prob[2], big, np.ones(8))
    A = mhd.Solver(n, prec="f32", stream=stream)
    A.set_state(s)
    cl.step(A)
    B = mhd.Solver(n, prec="f32", stream=stream)
    B.set_state(s)
    B.step_auto(0.7)
    assert cl.fallbacks() == 1
    assert np.array_equal(A.get_state(), B.get_state())
    # a tiny correction is applied
    cl.set_scales(prob[1], prob[2], np.full(8, 1e-6, dtype=np.float32), np.ones(8))
    cl.step(A)
    B.step_auto(0.7)
    assert cl.fallbacks() == 1
    assert not np.array_equal(A.get_state(), B.get_state())


def test_training_set_residual_and_statistics(env):
    """target = u_ref - u_plain bit for bit (one FP32 subtraction per value);
    the FP64 per-field sums against numpy's FP64 sums of the same values"""
    torch, mhd = env
    say("case: closure residual and statistics kernels")
    rng = np.random.default_rng(11)
    n = N3
    shape = (8, n[2], n[1], n[0])
    ur = rng.normal(1.0, 0.3, size=shape).astype(np.float32)
    up = (ur + rng.normal(0.0, 1e-2, size=shape)).astype(np.float32)
    cl = mhd.Closure(n)
    t = cl.residual(torch.from_numpy(ur).cuda(), torch.from_numpy(up).cuda())
    tn = t.cpu().numpy()
    assert np.array_equal(tn, ur - up)
    st = cl.stats(torch.from_numpy(up).cuda(), t)
    u64 = up.astype(np.float64).reshape(8, -1)
    t64 = tn.astype(np.float64).reshape(8, -1)
    ref = np.stack([u64.sum(1), (u64 * u64).sum(1), np.abs(u64).sum(1), np.abs(t64).sum(1)])
    assert np.allclose(st[:4], ref, rtol=1e-12, atol=0.0)


def _physical(u, gamma=5.0 / 3.0):
    """per-cell rho > 0 and p >= 0 (cell-centred field = mean of the faces),
    FP64, and the smallest pressure"""
    b = [0.5 * (u[5] + np.roll(u[5], -1, 2)), 0.5 * (u[6] + np.roll(u[6], -1, 1)),
         0.5 * (u[7] + np.roll(u[7], -1, 0))]
    p = (gamma - 1.0) * (u[4] - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]
                         - 0.5 * (b[0] ** 2 + b[1] ** 2 + b[2] ** 2))
    return bool((u[0] > 0).all() and (p >= 0).all()), float(p.min()), float(u[0].min())


def test_closure_step_scales_a_correction_down_to_stay_physical(env):
    """A correction that is non-physical at theta = 1 but clearly physical at
    theta = 1/2 is applied at 1/2: u_plain + fl(0.5 * delta) bit for bit."""
    torch, mhd = env
    say("case: closure guard levels")
    n = N3
    s = I.random_smooth(n, seed=8)
    prob = closure_problem(seed=2)
    stream = torch.cuda.current_stream()
    B = mhd.Solver(n, prec="f32", stream=stream)
    B.set_state(s)
    B.step_auto(0.7)
    ub = B.get_state_tensor().clone()
    plain = ub.cpu().numpy().astype(np.float64)
    cl = mhd.Closure(n, stream=stream)
    cl.set_params(C.flatten(C.init_params(3)).astype(np.float32))
    cl.set_scales(prob[1], prob[2], np.ones(8, dtype=np.float32), np.ones(8))
    d1 = cl.forward(ub).cpu().numpy().astype(np.float64)
    # the smallest scale t at which u + t d1 leaves the physical range
    lo, hi = 0.0, 1.0
    while _physical(plain + hi * d1)[0]:
        hi *= 2.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if _physical(plain + mid * d1)[0] else (lo, mid)
    sigma = 1.6 * hi
    ok1, pmin1, rmin1 = _physical(plain + sigma * d1)
    ok2, pmin2, rmin2 = _physical(plain + 0.5 * sigma * d1)
    say("t*", hi, "theta=1:", ok1, pmin1, rmin1, " theta=1/2:", ok2, pmin2, rmin2)
    assert not ok1 and ok2
    assert min(pmin1, rmin1) < -1e-3 and min(pmin2, rmin2) > 1e-3   # clear of FP32 rounding
    cl.set_scales(prob[1], prob[2], np.full(8, sigma, dtype=np.float32), np.ones(8))
    delta = cl.forward(ub).cpu().numpy()
    A = mhd.Solver(n, prec="f32", stream=stream)
    A.set_state(s)
    cl.step(A)
    got = A.get_state_tensor().cpu().numpy()
    want = ub.cpu().numpy() + np.float32(0.5) * delta
    assert cl.reduced() == 1 and cl.fallbacks() == 0
    assert np.array_equal(got, want)


def _roughness_means(u):
    """per-field mean of r_f = sum over axes |second difference| (numpy, FP64)"""
    U = u.reshape(8, N3[2], N3[1], N3[0])
    r = sum(np.abs(np.roll(U, -1, ax) - 2 * U + np.roll(U, 1, ax)) for ax in (1, 2, 3))
    return r.reshape(8, -1).mean(axis=1)


def test_gate_parity_and_roughness_statistics(env):
    """gate of the last forward against the oracle gate of the same FP32
    state (FP32 vs FP64 arithmetic: 1e-5 of the largest gate); the roughness
    row of the statistics kernel against numpy"""
    torch, mhd = env
    say("case: closure roughness gate")
    prob = closure_problem(seed=6)
    u = prob[0]
    R = _roughness_means(u) * np.linspace(0.5, 1.5, 8)
    cl = setup_closure(torch, mhd, prob)
    cl.set_gate(R)
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    cl.forward(ud)
    g = cl.gate().cpu().numpy().astype(np.float64)
    gr = C.gate(u.reshape(8, -1), R.astype(np.float32).astype(np.float64), N3)
    err = np.abs(g - gr).max() / gr.max()
    say("gate max rel err", err, "range", gr.min(), gr.max())
    assert err < 1e-5
    st = cl.stats(ud, ud)
    rsum = _roughness_means(u) * np.prod(N3)
    assert np.allclose(st[4], rsum, rtol=1e-12, atol=0.0)


def test_gated_network_forward_and_gradient_parity(env):
    torch, mhd = env
    say("case: gated closure network forward + gradient")
    prob = closure_problem(seed=7)
    u, mean, std, ps, out_scale, target, tscale = prob
    R = _roughness_means(u)
    cl = setup_closure(torch, mhd, prob)
    cl.set_gate(R)
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    td = torch.from_numpy(target.astype(np.float32).reshape(u.shape)).cuda()
    delta = cl.forward(ud).cpu().numpy().reshape(8, -1)
    gt = C.gate(u.reshape(8, -1), R.astype(np.float32).astype(np.float64), N3)
    x, psr, osc, tgt, ts = oracle_inputs(prob)
    ref = C.forward(x, psr, osc, N3, g=gt)
    e_fwd = np.linalg.norm(delta - ref) / np.linalg.norm(ref)
    L, g = cl.grad(ud, td)
    Lr, gr = C.loss_and_grad(x, psr, osc, tgt.astype(np.float64), ts, N3, g=gt)
    gr = C.flatten(gr)
    e_g = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    cos = float(np.dot(g, gr) / np.linalg.norm(g) / np.linalg.norm(gr))
    say("forward rel L2", e_fwd, "loss", L, Lr, "grad rel L2", e_g, "cos", cos)
    assert e_fwd < 3e-2
    assert L == pytest.approx(Lr, rel=1e-3)
    assert e_g < 3e-2 and cos > 0.999
    # switching the gate off restores the ungated correction
    cl.set_gate(None)
    d0 = cl.forward(ud).cpu().numpy().reshape(8, -1)
    ref0 = C.forward(x, psr, osc, N3)
    assert np.linalg.norm(d0 - ref0) / np.linalg.norm(ref0) < 3e-2


def test_consecutive_learned_steps_take_the_cfl_of_the_corrected_state(env):
    """a learned step changes the state after the plain step, so the next
    step cannot use the CFL maximum the plain step's last operator found:
    two learned steps in a row equal one learned step, a reload of its
    result into a fresh handle, and a second learned step, bit for bit"""
    torch, mhd = env
    say("case: closure steps and the fused CFL")
    n = N3
    s = I.random_smooth(n, seed=12)
    prob = closure_problem(seed=2)
    stream = torch.cuda.current_stream()
    cl = mhd.Closure(n, stream=stream)
    cl.set_params(C.flatten(C.init_params(3)).astype(np.float32))
    cl.set_scales(prob[1], prob[2], np.full(8, 3e-3, dtype=np.float32), np.ones(8))
    A = mhd.Solver(n, prec="f32", stream=stream)
    A.set_state(s)
    cl.step(A)
    cl.step(A)
    B = mhd.Solver(n, prec="f32", stream=stream)
    B.set_state(s)
    cl.step(B)
    mid = B.get_state_tensor().clone()
    Bb = mhd.Solver(n, prec="f32", stream=stream)
    Bb.set_state_tensor(mid)
    cl.step(Bb)
    assert cl.fallbacks() == 0
    a, b = A.get_state(), Bb.get_state()
    assert not np.array_equal(a, mid.cpu().numpy())
    assert np.array_equal(a, b)
