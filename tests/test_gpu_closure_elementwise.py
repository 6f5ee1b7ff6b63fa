"""Element-by-element parity of the whole closure network and of the Adam
step with the FP64 closure oracle.

The network test composes the oracle's layers (conv3d, project, gate,
project_T, dgrad, wgrad) and rounds the hidden activations and the
back-propagated gradients to BF16 at exactly the points where the kernels
store them (the input x, the ReLU outputs a1 and a2, the output gradient go
and the masked gradients g2 and g1); the rounding is done here, in the test,
not in the oracle.  What remains between the two is FP32 against FP64
accumulation and the rare BF16 rounding decision that the two accumulations
take differently.  Both act on the network output o, element by element
relative to its magnitude, and the correction is a fixed linear map of o
(fluid: s_f (o_f - mean o_f), at most 2 s_f max|o_f|; field: the discrete
curl of s_b (o_5, o_6, o_7), four terms of s_b o each).  Every element of the
correction is therefore compared with the composed reference within 1e-3
of that map's bound on its channel (2 s_f max|o_f| for a fluid channel,
4 s_b max|o_5..7| for a field channel): the mean removal and the curl
cancel most of o, so the correction's own largest value would be a scale
the rounding of o does not follow.  Every parameter gradient is compared
within 1e-3 of the largest gradient of its output channel (the weights
feeding that channel and its bias).

The Adam test gives the oracle's update (Kingma & Ba) the gradient the
library computed and compares the parameters after one and two training
steps element by element: FP32 rounding of the parameters (2 ulp) plus
1e-4 of the learning rate (the FP32 bias-correction factors 1 - beta^t).
"""
import sys

import numpy as np
import pytest

import bf16
from oracle import closure as C
from test_gpu_closure import N3, closure_problem, oracle_inputs, setup_closure, _roughness_means

pytestmark = pytest.mark.gpu

TOL = 1e-3


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1004_1680_amd import mhd
    mhd.load()
    return torch, mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def composed_forward(x, psr, osc, n, gt=None):
    """the network with BF16 hidden activations, as the kernels store them;
    also the projection's input (the gated output)"""
    w1, b1, w2, b2, w3, b3 = psr
    a1 = bf16.round(np.maximum(C.conv3d(x, w1, b1, n), 0.0))
    a2 = bf16.round(np.maximum(C.conv3d(a1, w2, b2, n), 0.0))
    o = C.conv3d(a2, w3, b3, n)
    og = o if gt is None else o * gt[:, None]
    d = C.project(og, osc, n)
    return d, a1, a2, og


def composed_grad(x, psr, osc, tgt, ts, n, gt=None):
    """the gradient of the loss with BF16 back-propagated gradients (go, g2,
    g1), as the kernels store them for their dgrad and wgrad inputs"""
    w1, b1, w2, b2, w3, b3 = psr
    d, a1, a2, og = composed_forward(x, psr, osc, n, gt)
    r = (d - tgt) / ts[:, None]
    gd = 2.0 * r / ts[:, None] / r.size
    go = C.project_T(gd, osc, n)
    if gt is not None:
        go = go * gt[:, None]
    gob = bf16.round(go)
    dw3, db3 = C.conv3d_wgrad(a2, gob, n, 32, 8)
    g2 = bf16.round(C.conv3d_dgrad(gob, w3, n) * (a2 > 0))
    dw2, db2 = C.conv3d_wgrad(a1, g2, n, 32, 32)
    g1 = bf16.round(C.conv3d_dgrad(g2, w2, n) * (a1 > 0))
    dw1, db1 = C.conv3d_wgrad(x, g1, n, 8, 32)
    return d, og, [dw1, db1, dw2, db2, dw3, db3]


def correction_errors(delta, ref, og, osc):
    """per channel: largest |delta - ref| over the projection's bound"""
    errs = []
    bmax = np.abs(og[:, 5:]).max()
    for f in range(8):
        bound = 2.0 * osc[f] * np.abs(og[:, f]).max() if f < 5 else 4.0 * osc[f] * bmax
        errs.append(float(np.abs(delta[f] - ref[f]).max() / bound))
    return errs


def gradient_errors(g, ref):
    """per layer and output channel: largest difference over the channel's
    largest reference gradient (weights and bias)"""
    errs = []
    parts = C.unflatten(g.astype(np.float64))
    for layer in range(3):
        dw, db = parts[2 * layer], parts[2 * layer + 1]
        rw, rb = ref[2 * layer], ref[2 * layer + 1]
        for co in range(rw.shape[2]):
            scale = max(np.abs(rw[:, :, co]).max(), abs(rb[co]))
            err = max(np.abs(dw[:, :, co] - rw[:, :, co]).max(), abs(db[co] - rb[co])) / scale
            errs.append((layer, co, float(err)))
    return errs


@pytest.mark.parametrize("gated", [False, True])
def test_network_elementwise(env, gated):
    torch, mhd = env
    say(f"case: closure network element by element, gate={gated}")
    prob = closure_problem(seed=7 if gated else 0)
    u, mean, std, ps, out_scale, target, tscale = prob
    cl = setup_closure(torch, mhd, prob)
    gt = None
    if gated:
        R = _roughness_means(u)
        cl.set_gate(R)
        gt = C.gate(u.reshape(8, -1), R.astype(np.float32).astype(np.float64), N3)
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    td = torch.from_numpy(target.astype(np.float32).reshape(u.shape)).cuda()
    delta = cl.forward(ud).cpu().numpy().reshape(8, -1).astype(np.float64)
    x, psr, osc, tgt, ts = oracle_inputs(prob)
    ref, og, gref = composed_grad(x, psr, osc, tgt.astype(np.float64), ts, N3, gt)
    ef = correction_errors(delta, ref, og, osc)
    L, g = cl.grad(ud, td)
    eg = gradient_errors(g, gref)
    worst = max(eg, key=lambda t: t[2])
    say("correction errors per channel (of the projection's bound):", [f"{e:.2e}" for e in ef])
    say("correction errors per channel (of the channel's largest value):",
        [f"{np.abs(delta[f] - ref[f]).max() / np.abs(ref[f]).max():.2e}" for f in range(8)])
    say(f"worst gradient error {worst[2]:.2e} (layer {worst[0]}, output channel {worst[1]})")
    assert max(ef) <= TOL, ef
    assert worst[2] <= TOL, worst


def test_adam_steps_match_the_oracle(env):
    torch, mhd = env
    say("case: Adam steps against the oracle")
    prob = closure_problem(seed=5)
    u, target = prob[0], prob[5]
    cl = setup_closure(torch, mhd, prob)
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    td = torch.from_numpy(target.astype(np.float32).reshape(u.shape)).cuda()
    lr = 1e-3
    p = cl.params().astype(np.float64)
    m = v = np.zeros_like(p)
    for t in (1, 2):
        _, g = cl.grad(ud, td)            # the gradient the training step uses
        cl.train_step(ud, td, lr, want_loss=False)
        got = cl.params().astype(np.float64)
        want, m, v = C.adam_step(p, g.astype(np.float64), m, v, t, lr)
        ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
        err = np.abs(got - want)
        bound = 2.0 * ulp + 1e-4 * lr
        say(f"t={t}: max |p - p_oracle| {err.max():.3e}, worst ratio to bound {(err / bound).max():.3f}, "
            f"max move {np.abs(want - p).max():.3e}")
        assert (err <= bound).all(), t
        p = got
