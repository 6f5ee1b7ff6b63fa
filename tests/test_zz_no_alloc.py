"""mhd_cfl_dt_noalloc, the CFL entry point that allocates nothing, against
mhd_cfl_dt on the same states: dt and vmax equal bit for bit (the same
kernels in the same order), on two calls in a row whose second grid is the
smaller, in both tiers; the records of a non-physical and of a static cold
state; a call captured in a HIP graph and replayed; argument checks."""
import sys

import numpy as np
import pytest

from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1004_1680_amd import mhd
    mhd.load()
    return torch, mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference(mhd, s, n, prec):
    """dt, vmax and the error class of mhd_cfl_dt on a handle"""
    S = mhd.Solver(n, prec=prec)
    S.set_state(s)
    try:
        dt = S.cfl_dt(0.7)
        out = (dt, S.relaxation_speed(), 0)
    except mhd.NonPhysicalState:
        out = (0.0, 0.0, 1)
    except mhd.MHDError:
        out = (0.0, 0.0, 2)
    S.close()
    return out


def device_state(torch, s, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(s)).to(device="cuda", dtype=dt).reshape(-1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_cfl_equals_the_handle_cfl(env, prec):
    torch, mhd = env
    big, small = (48, 32, 40), (16, 16, 16)
    for n, seed in ((big, 3), (small, 4)):      # the second call has the smaller input
        say(f"case: noalloc CFL {n} {prec}")
        s = I.random_smooth(n, seed=seed)
        if prec == "f32":
            s = s.astype(np.float32).astype(np.float64)
        t = device_state(torch, s, prec)
        out = mhd.cfl_dt_noalloc(t, n, cfl=0.7)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = reference(mhd, s, n, prec)
        say("noalloc", got, "handle", ref)
        assert got[0] == ref[0] and got[1] == ref[1] and got[2] == 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_cfl_records(env, prec):
    torch, mhd = env
    n = (16, 12, 8)
    bad = I.random_smooth(n, seed=5)
    bad[4, 3, 5, 7] = -1.0                     # negative energy: p < 0
    cold = np.zeros((8,) + n[::-1])
    cold[0] = 1.0                              # p = 0, b = 0, v = 0: no signal speed
    good = I.random_smooth(n, seed=6)
    out = None
    for s, rec in ((bad, 1), (cold, 2), (good, 0)):
        out = mhd.cfl_dt_noalloc(device_state(torch, s, prec), n, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = reference(mhd, s, n, prec)
        say("record", got, ref)
        assert got[2] == rec == ref[2]
        if rec:
            assert got[0] == 0.0 and got[1] == 0.0
        else:
            assert got[0] == ref[0] and got[1] == ref[1]


def test_noalloc_cfl_in_a_graph(env):
    """captured once, replayed three times on changed state contents, with
    eager calls and synchronisations in between: every replay equals the
    eager call on the same contents"""
    torch, mhd = env
    n = (32, 16, 24)
    s = I.random_smooth(n, seed=7)
    t = device_state(torch, s, "f32")
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    mhd.cfl_dt_noalloc(t, n, out=out)          # the first call on the device looks the array up
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        mhd.cfl_dt_noalloc(t, n, out=out, stream=torch.cuda.current_stream())
    for rep in range(3):
        s2 = I.random_smooth(n, seed=20 + rep)
        t.copy_(device_state(torch, s2, "f32"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        eager = mhd.cfl_dt_noalloc(t, n).cpu().numpy()
        say("replay", rep, got, eager)
        assert np.array_equal(got, eager)
        assert got[0] > 0 and got[2] == 0


def test_noalloc_cfl_argument_checks(env):
    torch, mhd = env
    t = torch.zeros(8 * 16 ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        mhd.cfl_dt_noalloc(t, (16, 16, 8))                     # size mismatch (binding)
    lib = mhd.load()
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    p, o = mhd._dptr(t), mhd._dptr(out)
    assert lib.mhd_cfl_dt_noalloc(p, 16, 16, 10, 0, 5.0 / 3.0, 0.7, o, None) == mhd.MHD_EINVAL
    assert lib.mhd_cfl_dt_noalloc(p, 2048, 16, 16, 0, 5.0 / 3.0, 0.7, o, None) == mhd.MHD_EINVAL
    assert lib.mhd_cfl_dt_noalloc(None, 16, 16, 16, 0, 5.0 / 3.0, 0.7, o, None) == mhd.MHD_EINVAL
    assert lib.mhd_cfl_dt_noalloc(p, 16, 16, 16, 2, 5.0 / 3.0, 0.7, o, None) == mhd.MHD_EINVAL
    assert lib.mhd_cfl_dt_noalloc(p, 16, 16, 16, 0, 1.0, 0.7, o, None) == mhd.MHD_EINVAL
    assert lib.mhd_cfl_dt_noalloc(p, 16, 16, 16, 0, 5.0 / 3.0, 0.0, o, None) == mhd.MHD_EINVAL
    assert "cfl" in mhd.last_error()
