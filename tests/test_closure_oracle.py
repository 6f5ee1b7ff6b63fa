"""Pins of the closure oracle: the convolution against an independent
roll-based evaluation, dgrad/wgrad against the adjoint identities they must
satisfy, the projection against the invariants it exists for (no change of
any total, zero discrete div b) and its adjoint, and the full gradient
against central finite differences."""
import numpy as np
import pytest

from oracle import closure as C


def roll_conv(x, w, b, n):
    """y = b + sum_o shift(x, d(o)) @ w[o], with numpy rolls on the grid"""
    nx, ny, nz = n
    X = x.reshape(nz, ny, nx, -1)
    y = np.zeros((nz, ny, nx, w.shape[2])) + (0 if b is None else b)
    for o in range(27):
        dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
        S = np.roll(X, shift=(-dz, -dy, -dx), axis=(0, 1, 2))   # S[c] = X[c + d]
        y += S @ w[o]
    return y.reshape(nx * ny * nz, -1)


N3 = (8, 4, 6)


@pytest.mark.parametrize("cin,cout", [(8, 32), (32, 32), (32, 8)])
def test_conv_matches_roll_evaluation(cin, cout):
    rng = np.random.default_rng(cin + cout)
    N = np.prod(N3)
    x = rng.normal(size=(N, cin))
    w = rng.normal(size=(27, cin, cout))
    b = rng.normal(size=cout)
    assert np.allclose(C.conv3d(x, w, b, N3), roll_conv(x, w, b, N3), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("cin,cout", [(8, 32), (32, 8)])
def test_dgrad_and_wgrad_are_adjoints(cin, cout):
    rng = np.random.default_rng(7)
    N = np.prod(N3)
    x = rng.normal(size=(N, cin))
    dy = rng.normal(size=(N, cout))
    w = rng.normal(size=(27, cin, cout))
    # <conv(x; w), dy> = <x, dgrad(dy; w)> = <wgrad(x, dy), w>
    lhs = np.sum(C.conv3d(x, w, None, N3) * dy)
    assert np.sum(x * C.conv3d_dgrad(dy, w, N3)) == pytest.approx(lhs, rel=1e-12)
    dw, db = C.conv3d_wgrad(x, dy, N3, cin, cout)
    assert np.sum(dw * w) == pytest.approx(lhs, rel=1e-12)
    assert np.allclose(db, dy.sum(axis=0), rtol=1e-12)


def test_projection_keeps_totals_and_div_b():
    rng = np.random.default_rng(3)
    n = (8, 12, 4)
    N = np.prod(n)
    o = rng.normal(size=(N, 8))
    sc = rng.uniform(0.5, 2.0, 8)
    d = C.project(o, sc, n)
    assert np.all(np.abs(d[:5].sum(axis=1)) < 1e-12 * np.abs(d[:5]).sum(axis=1))
    bx, by, bz = (d[5 + k].reshape(n[2], n[1], n[0]) for k in range(3))
    div = (np.roll(bx, -1, 2) - bx) + (np.roll(by, -1, 1) - by) + (np.roll(bz, -1, 0) - bz)
    assert np.abs(div).max() < 1e-12 * np.abs(d[5:]).max()
    # adjoint: <project(o), g> = <o, project_T(g)>
    g = rng.normal(size=(8, N))
    assert np.sum(d * g) == pytest.approx(np.sum(o * C.project_T(g, sc, n)), rel=1e-12)


def test_gradient_matches_finite_differences():
    n = (8, 8, 4)
    N = np.prod(n)
    rng = np.random.default_rng(0)
    x = rng.normal(size=(N, 8))
    ps = C.init_params(1)
    sc = rng.uniform(0.5, 1.5, 8)
    t = rng.normal(size=(8, N))
    ts = rng.uniform(0.5, 2.0, 8)
    L, g = C.loss_and_grad(x, ps, sc, t, ts, n)
    v, gv = C.flatten(ps), C.flatten(g)
    assert v.size == 41544
    for idx in (3, 500, 6950, 7000, 20000, 34000, 41000):
        e = 1e-6
        vp, vm = v.copy(), v.copy()
        vp[idx] += e
        vm[idx] -= e
        Lp, _ = C.loss_and_grad(x, C.unflatten(vp), sc, t, ts, n)
        Lm, _ = C.loss_and_grad(x, C.unflatten(vm), sc, t, ts, n)
        fd = (Lp - Lm) / (2 * e)
        assert gv[idx] == pytest.approx(fd, rel=1e-5, abs=1e-11), idx


def test_gate_vanishes_on_linear_and_uniform_states():
    """second differences of a uniform state are zero; along a periodic axis
    a linear profile is impossible, but a profile linear within the interior
    gives nonzero r only next to its wrap-around jump"""
    n = (8, 6, 4)
    N = np.prod(n)
    u = np.ones((8, N)) * np.arange(1, 9)[:, None]
    assert np.all(C.gate(u, np.ones(8), n) == 0.0)
    # u_0 = i (x index): r_0 = |jump terms| only at i = 0 and i = nx - 1
    i = np.arange(N) % n[0]
    u = np.zeros((8, N))
    u[0] = i
    g = C.gate(u, np.ones(8), n).reshape(n[2], n[1], n[0])
    # g0 at i = 0: |1 - 0 + (nx - 1)| ... = |u(1) - 2u(0) + u(nx-1)| = nx;
    # at i = nx - 1: |u(0) - 2(nx-1) + u(nx-2)| = nx; elsewhere 0; / 8
    g0 = np.zeros(n[0])
    g0[0] = g0[-1] = n[0] / 8.0
    want = np.maximum.reduce([g0, np.roll(g0, 1), np.roll(g0, -1)])
    assert np.array_equal(g, np.broadcast_to(want, g.shape))


def test_gate_of_a_sine_matches_its_closed_form():
    """u_f = sin(2 pi k x_i / nx): second difference = -4 sin^2(pi k / nx) u;
    g0 = (1/8) sum_f r_f / R_f, then the max over the 7-point stencil"""
    n = (16, 4, 4)
    N = np.prod(n)
    i = np.arange(N) % n[0]
    k = 3
    u = np.zeros((8, N))
    R = np.arange(1.0, 9.0)
    for f in (1, 4, 6):
        u[f] = (f + 1) * np.sin(2 * np.pi * k * i / n[0])
    s2 = 4 * np.sin(np.pi * k / n[0]) ** 2
    g0 = sum((f + 1) * s2 * np.abs(np.sin(2 * np.pi * k * np.arange(n[0]) / n[0])) / R[f]
             for f in (1, 4, 6)) / 8.0
    want = np.maximum.reduce([g0, np.roll(g0, 1), np.roll(g0, -1)])
    g = C.gate(u, R, n).reshape(n[2], n[1], n[0])
    assert np.allclose(g, np.broadcast_to(want, g.shape), rtol=1e-12, atol=1e-14)


def test_gate_spreads_one_point_to_its_face_neighbours():
    n = (6, 5, 7)
    N = np.prod(n)
    u = np.zeros((8, N))
    u[3].reshape(n[2], n[1], n[0])[2, 2, 2] = 1.0
    g = C.gate(u, np.ones(8), n).reshape(n[2], n[1], n[0])
    # g0: 6/8 at the point (three axes, |-2| each), 1/8 at its 6 neighbours
    assert g[2, 2, 2] == 6 / 8
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        assert g[2 + d[0], 2 + d[1], 2 + d[2]] == 6 / 8
    # cells two faces away and the 12 edge-diagonal cells see a neighbour's 1/8
    assert g[2, 2, 4] == 1 / 8 and g[2, 3, 3] == 1 / 8
    assert g[5, 2, 2] == 0.0
    assert np.count_nonzero(g) == 1 + 6 + 6 + 12


def test_gated_gradient_matches_finite_differences():
    n = (8, 8, 4)
    N = np.prod(n)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(N, 8))
    ps = C.init_params(2)
    sc = rng.uniform(0.5, 1.5, 8)
    t = rng.normal(size=(8, N))
    ts = rng.uniform(0.5, 2.0, 8)
    g = rng.uniform(0.0, 2.0, N)
    L, gr = C.loss_and_grad(x, ps, sc, t, ts, n, g=g)
    v, gv = C.flatten(ps), C.flatten(gr)
    for idx in (3, 6950, 20000, 41000, 41540):
        e = 1e-6
        vp, vm = v.copy(), v.copy()
        vp[idx] += e
        vm[idx] -= e
        Lp, _ = C.loss_and_grad(x, C.unflatten(vp), sc, t, ts, n, g=g)
        Lm, _ = C.loss_and_grad(x, C.unflatten(vm), sc, t, ts, n, g=g)
        assert gv[idx] == pytest.approx((Lp - Lm) / (2 * e), rel=1e-5, abs=1e-11), idx
    # the gate multiplies the network output before the projection
    d = C.forward(x, ps, sc, n, g=g)
    _, (_, _, _, o) = C.forward(x, ps, sc, n, keep=True)
    assert np.allclose(d, C.project(o * g[:, None], sc, n), rtol=1e-13, atol=1e-15)


# --- Adam (the optimizer of the training step) -------------------------------

def test_adam_first_step_closed_form():
    """at t = 1 the bias corrections give m_hat = g and v_hat = g^2, so every
    parameter moves by -lr g / (|g| + eps), whatever the betas"""
    rng = np.random.default_rng(11)
    p = rng.normal(size=1000)
    g = rng.normal(size=1000) * 10.0 ** rng.uniform(-9, 2, 1000)
    z = np.zeros(1000)
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9)):
        q, m, v = C.adam_step(p, g, z, z, 1, 1e-3, b1, b2)
        assert np.allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
        assert np.allclose(m, (1 - b1) * g, rtol=1e-15, atol=0)
        assert np.allclose(v, (1 - b2) * g * g, rtol=1e-15, atol=0)


def test_adam_constant_and_alternating_gradients():
    """a constant gradient keeps m_hat = g and v_hat = g^2 at every step (the
    bias corrections exactly undo the zero start); after g, a gradient -g
    gives at t = 2 m = beta1 (1-beta1) g - (1-beta1) g = -(1-beta1)^2 g,
    m_hat = -(1-beta1)^2 g / (1 - beta1^2) = -g (1-beta1)/(1+beta1) = -g/19
    and v_hat = g^2, so the second move is +lr g / (19 (|g| + eps))"""
    rng = np.random.default_rng(12)
    p0 = rng.normal(size=200)
    g = rng.normal(size=200)
    lr = 2e-3
    p, m, v = p0, np.zeros(200), np.zeros(200)
    for t in range(1, 6):
        p, m, v = C.adam_step(p, g, m, v, t, lr)
        assert np.allclose(p, p0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14), t
    p, m, v = C.adam_step(p0, g, np.zeros(200), np.zeros(200), 1, lr)
    q, m, v = C.adam_step(p, -g, m, v, 2, lr)
    assert np.allclose(q - p, lr * g / (19.0 * (np.abs(g) + 1e-8)), rtol=0, atol=1e-15)


def test_adam_zero_gradient_and_scale_invariance():
    """zero gradient: no move; without eps the move does not depend on the
    gradient's scale (Adam divides by the root mean square)"""
    rng = np.random.default_rng(13)
    p = rng.normal(size=100)
    z = np.zeros(100)
    q, _, _ = C.adam_step(p, z, z, z, 1, 1e-3)
    assert np.array_equal(q, p)
    g1, g2 = rng.normal(size=100), rng.normal(size=100)
    a, m, v = C.adam_step(p, g1, z, z, 1, 1e-3, eps=0.0)
    a, _, _ = C.adam_step(a, g2, m, v, 2, 1e-3, eps=0.0)
    b, m, v = C.adam_step(p, 37.0 * g1, z, z, 1, 1e-3, eps=0.0)
    b, _, _ = C.adam_step(b, 37.0 * g2, m, v, 2, 1e-3, eps=0.0)
    assert np.allclose(a, b, rtol=0, atol=1e-15)
