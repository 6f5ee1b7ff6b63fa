"""FP64 oracle of the learned closure (test infrastructure only).

The closure corrects one plain coarse step: x = (u_plain - mean) / std per
channel -> conv(8->32) -> ReLU -> conv(32->32) -> ReLU -> conv(32->8) -> the
conservative projection (mean-free fluid corrections, discrete curl of an
edge potential for b) -> delta, and u = u_plain + delta.  Convolutions are
periodic 3x3x3 with channel-last activations; the loss is the mean squared
error of delta against the target correction, each channel divided by its
target scale.  With a roughness gate g(u) (gate()), the projection acts on
g * o, cell by cell.  Everything here is plain FP64 (C loops in
closure_oracle.c, composed in numpy).
"""
import ctypes

import numpy as np

from .oracle import load

CH = (8, 32, 32, 8)


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def conv3d(x, w, b, n):
    """x[cell][cin], w[27][cin][cout], b[cout] -> y[cell][cout]"""
    x, w = _c(x), _c(w)
    cin, cout = w.shape[1], w.shape[2]
    y = np.empty((x.shape[0], cout))
    bb = _c(b) if b is not None else None
    load().oracle_conv3d(n[0], n[1], n[2], cin, cout, _p(x), _p(w),
                         _p(bb) if bb is not None else None, _p(y))
    return y


def conv3d_dgrad(dy, w, n):
    dy, w = _c(dy), _c(w)
    cin, cout = w.shape[1], w.shape[2]
    dx = np.empty((dy.shape[0], cin))
    load().oracle_conv3d_dgrad(n[0], n[1], n[2], cin, cout, _p(dy), _p(w), _p(dx))
    return dx


def conv3d_wgrad(x, dy, n, cin, cout):
    x, dy = _c(x), _c(dy)
    dw = np.empty((27, cin, cout))
    db = np.empty(cout)
    load().oracle_conv3d_wgrad(n[0], n[1], n[2], cin, cout, _p(x), _p(dy), _p(dw), _p(db))
    return dw, db


def project(o, scale, n):
    """o[cell][8] -> delta[8][cell] (field-major)"""
    o, sc = _c(o), _c(scale)
    d = np.empty((8, o.shape[0]))
    load().oracle_closure_project(n[0], n[1], n[2], _p(o), _p(sc), _p(d))
    return d


def project_T(g, scale, n):
    g, sc = _c(g), _c(scale)
    go = np.empty((g.shape[1], 8))
    load().oracle_closure_project_T(n[0], n[1], n[2], _p(g), _p(sc), _p(go))
    return go


def gate(u, R, n):
    """u[8][cell] (field-major state), R[8] > 0 -> g[cell]"""
    u, R = _c(u).reshape(8, -1), _c(R)
    g = np.empty(u.shape[1])
    load().oracle_closure_gate(n[0], n[1], n[2], _p(u), _p(R), _p(g))
    return g


def init_params(seed=0):
    """He-normal weights, zero biases (w[27][cin][cout] per layer)."""
    rng = np.random.default_rng(seed)
    ps = []
    for cin, cout in zip(CH[:-1], CH[1:]):
        ps.append(rng.normal(0.0, np.sqrt(2.0 / (27 * cin)), size=(27, cin, cout)))
        ps.append(np.zeros(cout))
    ps[-2] *= 0.1                       # start near the plain step
    return ps


def flatten(ps):
    return np.concatenate([p.ravel() for p in ps])


def unflatten(v):
    ps, k = [], 0
    for cin, cout in zip(CH[:-1], CH[1:]):
        ps.append(v[k:k + 27 * cin * cout].reshape(27, cin, cout)); k += 27 * cin * cout
        ps.append(v[k:k + cout]); k += cout
    return ps


def normalize(u, mean, std):
    """state u[8][cell] (field-major) -> x[cell][8]"""
    return ((u - mean[:, None]) / std[:, None]).T.copy()


def forward(x, ps, scale, n, keep=False, g=None):
    """x[cell][8] -> delta[8][cell]; with keep, also the activations; g:
    the roughness gate per cell (None: no gate)"""
    w1, b1, w2, b2, w3, b3 = ps
    z1 = conv3d(x, w1, b1, n)
    a1 = np.maximum(z1, 0.0)
    z2 = conv3d(a1, w2, b2, n)
    a2 = np.maximum(z2, 0.0)
    o = conv3d(a2, w3, b3, n)
    d = project(o if g is None else o * g[:, None], scale, n)
    if keep:
        return d, (x, a1, a2, o)
    return d


def loss_and_grad(x, ps, scale, target, tscale, n, g=None):
    """L = mean over channels and cells of ((delta - target)/tscale)^2 and
    its gradient with respect to every parameter (g: roughness gate)"""
    d, (x0, a1, a2, o) = forward(x, ps, scale, n, keep=True, g=g)
    r = (d - target) / tscale[:, None]
    L = float(np.mean(r * r))
    gd = 2.0 * r / tscale[:, None] / r.size
    go = project_T(gd, scale, n)
    if g is not None:
        go = go * g[:, None]
    w1, b1, w2, b2, w3, b3 = ps
    dw3, db3 = conv3d_wgrad(a2, go, n, 32, 8)
    g2 = conv3d_dgrad(go, w3, n) * (a2 > 0)
    dw2, db2 = conv3d_wgrad(a1, g2, n, 32, 32)
    g1 = conv3d_dgrad(g2, w2, n) * (a1 > 0)
    dw1, db1 = conv3d_wgrad(x0, g1, n, 8, 32)
    return L, [dw1, db1, dw2, db2, dw3, db3]


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) of parameters p with
    gradient g at step t >= 1, from the first- and second-moment estimates
    m, v of the previous step (zeros before the first).  Returns (p, m, v):
        m <- beta1 m + (1 - beta1) g,     v <- beta2 v + (1 - beta2) g^2,
        p <- p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
