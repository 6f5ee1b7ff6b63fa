"""The visit order of the x sweeps' row tiles (groups of rows along y, one
group per z in turn) is a launch-shape choice: steps come out the same bit
for bit for every group size, the linear order included, on grids where the
groups hold one or several tiles and where the rows of a workgroup do not
divide ny (linear order)."""
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


def steps(M, s, n, prec, group, nsteps=2):
    S = M.Solver(n, prec=prec)
    S.set_launch(M.MHD_TUNE_ROW_GROUP, group)
    rows = S.launch(M.MHD_TUNE_ROW_GROUP)
    S.set_state(s)
    for _ in range(nsteps):
        S.step_auto(0.7)
    assert S.status() == nsteps
    out = S.get_state(), S.time()
    S.close()
    return out, rows


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n", [(64, 128, 24), (32, 96, 16), (16, 128, 12), (40, 28, 8)])
def test_row_order_does_not_change_steps(M, n, prec):
    say(f"case: row order n={n} {prec}")
    s = I.random_smooth(n, seed=51, amp_b=0.15 * n[1] / n[0] if n[1] < n[0] else 0.15)
    (ref, tref), rows = steps(M, s, n, prec, n[1])
    assert rows == n[1]
    seen = set()
    for g in (0, 1, 16, 32, 1000):
        (out, t), rows = steps(M, s, n, prec, g)
        seen.add(rows)
        assert np.array_equal(out, ref) and t == tref, (g, rows)
    say("rows per group seen", sorted(seen))


def test_row_group_resolution(M):
    # 64 x 128 x 24: 16 rows per workgroup, 8 tiles per y line
    S = M.Solver((64, 128, 24), prec="f32")
    assert S.launch(M.MHD_TUNE_ROW_GROUP) == 64          # built-in: 64 rows
    S.set_launch(M.MHD_TUNE_ROW_GROUP, 40)
    assert S.launch(M.MHD_TUNE_ROW_GROUP) == 32          # largest divisor of 8 tiles within 40 rows
    S.set_launch(M.MHD_TUNE_ROW_GROUP, 8)
    assert S.launch(M.MHD_TUNE_ROW_GROUP) == 128         # below one workgroup's rows: linear
    with pytest.raises(M.MHDError):
        S.set_launch(M.MHD_TUNE_ROW_GROUP, -1)
    S.close()
    # 40 x 28 x 8: 25 rows per workgroup do not divide 28
    S = M.Solver((40, 28, 8), prec="f32")
    assert S.launch(M.MHD_TUNE_ROW_GROUP) == 28
    S.close()
