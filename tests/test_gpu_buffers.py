"""Caller-owned state buffers (mhd_create_ex with dev_buf_a, dev_buf_b):
steps give the same states bit for bit as with the library's own buffers,
the state lives in the caller's memory, the handle never frees it, and the
conditions the runtime can check are refused with MHD_EINVAL."""
import sys

import numpy as np
import pytest

from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1004_1680_amd import mhd
    mhd.load()
    return mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_caller_buffers_step_like_own_buffers(M, prec):
    import torch
    n = (24, 16, 32)
    ncell = n[0] * n[1] * n[2]
    say(f"case: caller-owned buffers {n} {prec}")
    dt = torch.float32 if prec == "f32" else torch.float64
    a = torch.full((8 * ncell,), 7.0, dtype=dt, device="cuda")
    b = torch.full((8 * ncell + 64,), 7.0, dtype=dt, device="cuda")   # longer is fine
    s = I.random_smooth(n, seed=41)
    outs = []
    for bufs in ((a, b), None):
        S = M.Solver(n, prec=prec, buffers=bufs)
        S.set_state(s)
        for _ in range(3):
            S.step_auto(0.7)
        assert S.status() == 3
        outs.append((S.get_state(), S.time()))
        if bufs is not None:
            # every field of the state sits in one of the caller's buffers
            fa = a.view(8, ncell).cpu().numpy().astype(np.float64)
            fb = b[:8 * ncell].view(8, ncell).cpu().numpy().astype(np.float64)
            g = outs[-1][0].reshape(8, ncell)
            for f in range(8):
                assert np.array_equal(g[f], fa[f]) or np.array_equal(g[f], fb[f]), f
        S.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    # closing the handle left the caller's memory alone
    a.fill_(1.5)
    b.fill_(2.5)
    torch.cuda.synchronize()
    assert float(a.sum()) == 1.5 * a.numel() and float(b.sum()) == 2.5 * b.numel()


def test_caller_buffer_checks(M):
    import torch
    n = (16, 16, 16)
    ncell = 16 ** 3
    say("case: caller-owned buffer checks")
    g = 5.0 / 3.0
    c = torch.zeros(2 * 8 * ncell + 256, dtype=torch.float32, device="cuda")
    p = c.data_ptr()
    assert p % 256 == 0
    lib = M.load()
    # misaligned
    assert not lib.mhd_create_ex(*n, g, M.MHD_F32, None, p + 4, p + 4 * 8 * ncell + 256)
    assert "aligned" in M.last_error()
    # overlapping
    assert not lib.mhd_create_ex(*n, g, M.MHD_F32, None, p, p + 256)
    assert "overlap" in M.last_error()
    # host memory
    h = np.zeros(8 * ncell + 64, dtype=np.float32)
    hp = (h.ctypes.data + 255) // 256 * 256
    assert not lib.mhd_create_ex(*n, g, M.MHD_F32, None, hp, p)
    assert "memory" in M.last_error()
    # adjacent, non-overlapping halves of one allocation are accepted
    h1 = lib.mhd_create_ex(*n, g, M.MHD_F32, None, p, p + 4 * 8 * ncell + 256)
    assert h1
    lib.mhd_destroy(h1)
    # the binding checks tensors before the call
    with pytest.raises(ValueError):
        M.Solver(n, prec="f32", buffers=(c[:8 * ncell - 1], c[8 * ncell:]))
    with pytest.raises(ValueError):
        M.Solver(n, prec="f64", buffers=(c, c))
    torch.cuda.synchronize()
