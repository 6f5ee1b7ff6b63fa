"""Parity at the full benchmark sizes (512^3 and 1024^3 FP32 Orszag-Tang-type
states, the launch configuration bench.py times), on sampled outputs.

One step of the whole grid runs on the GPU.  The FP64 oracle cannot step a
1024^3 grid in test time, but one step only reaches 16 cells along any axis:
the oracle steps 32 periodic 40^3 windows cut from the same float-rounded
initial state with the GPU's dt and relaxation speed (dt scaled by n / 40,
since the scheme's grid spacing is 1 / nx), and the 8^3 interior of each
window must equal the full-grid result (checked exactly for the oracle
against its own full-grid step in test_window_margin_is_exact below, on the
CPU).  Interiors are compared with the FP32 tolerance of the other tests
(1e-5 of each field family's largest magnitude in the samples; 1e-12 for the FP64 tier).  Windows
include ones that wrap around the periodic boundary.  Properties that hold
at any size are checked on the whole grid: conserved totals (FP64 sums) and
div b."""
import sys

import numpy as np
import pytest

import oracle
from paper_1004_1680_amd import inputs as I

MARGIN, INNER = 16, 8
W = 2 * MARGIN + INNER
FAMILIES = ([0], [1, 2, 3], [4], [5, 6, 7])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def window_index(n, center):
    """periodic index arrays (z, y, x) of the W^3 window around center"""
    return [(np.arange(W) + center[d] - W // 2) % n[d] for d in (2, 1, 0)]


def cut(a, idx):
    return a[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]


TOL = {"f32": 1e-5, "f64": 1e-12}


@pytest.mark.gpu
@pytest.mark.parametrize("n,prec", [(512, "f32"), (1024, "f32"), (512, "f64")])
def test_full_size_sampled_parity(n, prec):
    import torch
    from paper_1004_1680_amd import mhd
    mhd.load()
    say(f"case: {n}^3 {prec} Orszag-Tang, one step, sampled windows")
    N = (n, n, n)
    stream = torch.cuda.current_stream()
    S = mhd.Solver(N, prec=prec, stream=stream)
    u0 = I.orszag_tang_torch(N, seed=0, dtype=torch.float64 if prec == "f64" else torch.float32)
    S.set_state_tensor(u0)
    d0 = S.diag()
    dt = S.cfl_dt(0.7)
    c = S.relaxation_speed()
    S.step_auto(0.7)                     # the benchmark's step: device CFL + 12 operators
    S.status()
    d1 = S.diag()
    u1 = S.get_state_tensor()
    say("dt", dt, "c", c)
    # fixed windows (periodic wraps on every axis), windows across the
    # launch-shape seams (64-row groups of the x sweeps' tile order; march
    # chunk boundaries at multiples of 64 along y and z) and seeded random
    # ones: 32 windows, 16384 sampled cells
    centers = [(n // 2, n // 3, n // 5), (0, 0, 0), (n - 3, 7, n // 2), (n // 4, n - 1, 3),
               (5 * n // 8, 3 * n // 4, n - 9), (n // 7, n // 2, 2 * n // 3),
               (n // 3, 64, n // 2), (n // 5, 127, 3 * n // 4), (2 * n // 3, n // 2, 256 % n),
               (n - 1, 191, 255 % n), (17, 320 % n, 64), (n // 2, n // 2 + 1, 128)]
    rng = np.random.default_rng(2024)
    centers += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(20)]
    err = np.zeros(4)
    scale = np.zeros(4)
    for ctr in centers:
        idx = window_index(N, ctr)
        ti = [torch.as_tensor(v, device="cuda") for v in idx]
        w0 = u0.index_select(1, ti[0]).index_select(2, ti[1]).index_select(3, ti[2]).double().cpu().numpy()
        w1 = u1.index_select(1, ti[0]).index_select(2, ti[1]).index_select(3, ti[2]).double().cpu().numpy()
        ref = oracle.step(np.ascontiguousarray(w0), dt * n / W, c)
        sl = (slice(None),) + (slice(MARGIN, MARGIN + INNER),) * 3
        a, b = w1[sl], ref[sl]
        for q, fam in enumerate(FAMILIES):
            err[q] = max(err[q], np.abs(a[fam] - b[fam]).max())
            scale[q] = max(scale[q], np.abs(b[fam]).max())
    rel = err / scale
    say("family rel err (rho, m, e, b)", rel)
    assert np.all(rel <= TOL[prec])
    # whole-grid properties: totals to FP32 rounding, div b stays at rounding
    tot_rel = np.abs(d1[:8] - d0[:8]) / np.maximum(np.abs(d0[:8]), 1e-30)
    say("total changes", tot_rel[:5], "div b", d0[8], d1[8])
    for f, r in enumerate(tot_rel[:5]):
        if abs(d0[f]) > 1e-6:
            assert r < 1e-5, (f, r)
    assert d1[8] < 1e-5
    S.close()


def test_window_margin_is_exact():
    """the oracle's step of a periodic W^3 window equals its full-grid step
    on the INNER^3 interior, bit for bit (margin = dependency reach of one
    step), on a state with structure along every axis"""
    oracle.load()
    n = (96, 96, 96)
    rs = I.random_smooth(n, seed=3)
    s = I.orszag_tang(n) + 0.02 * (rs - rs.mean(axis=(1, 2, 3), keepdims=True))
    dt, c = oracle.cfl(s)
    full = oracle.step(s, dt, c)
    sl = (slice(None),) + (slice(MARGIN, MARGIN + INNER),) * 3
    for ctr in [(5, 7, 9), (50, 60, 70), (95, 0, 48)]:
        idx = window_index(n, ctr)
        out = oracle.step(np.ascontiguousarray(cut(s, idx)), dt * n[0] / W, c)
        assert np.array_equal(out[sl], cut(full, idx)[sl]), ctr
