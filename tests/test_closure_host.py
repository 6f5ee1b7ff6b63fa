"""Host-side logic of the closure training driver (no GPU): the relative
L1 error of the evaluation, the equal-L1 wall-time interpolation between
plain resolutions, and the initial parameters."""
import numpy as np
import pytest

from paper_1004_1680_amd import closure_train as CT


def test_l1_rel_definition():
    rng = np.random.default_rng(3)
    b = rng.normal(size=(8, 4, 4, 4)) + 2.0
    assert CT.l1_rel(b, b) == 0.0
    a = b.copy()
    a[0] += 0.1                      # density off by 0.1 everywhere
    want = 0.1 / np.mean(np.abs(b[0])) / 8
    assert CT.l1_rel(a, b) == pytest.approx(want, rel=1e-12)


def test_l1_rel_zero_field_takes_its_family_scale():
    b = np.ones((8, 2, 2, 2))
    b[3] = 0.0                       # m_z identically zero: family (m_x, m_y, m_z)
    a = b.copy()
    a[3] = 0.5
    fam = np.mean(np.abs(b[[1, 2, 3]]))
    assert CT.l1_rel(a, b) == pytest.approx(0.5 / fam / 8, rel=1e-12)


def test_equal_l1_wall_is_log_log_interpolation():
    plains = [(1e-1, 0.01), (1e-2, 1.0), (1e-3, 100.0)]
    # the geometric mean of two bracketing errors lands on the geometric
    # mean of their wall times
    assert CT._equal_l1_wall(plains, np.sqrt(1e-1 * 1e-2)) == pytest.approx(0.1, rel=1e-12)
    assert CT._equal_l1_wall(plains, 1e-2) == pytest.approx(1.0, rel=1e-12)
    assert CT._equal_l1_wall(plains, np.sqrt(1e-2 * 1e-3)) == pytest.approx(10.0, rel=1e-12)
    assert CT._equal_l1_wall(plains, 0.5) is None          # worse than the coarsest
    assert CT._equal_l1_wall(plains, 1e-4) is None         # better than the finest
    assert CT._equal_l1_wall([(1e-2, 1.0)], 1e-2) is None  # one resolution brackets nothing


def test_initial_parameters():
    p = CT.init_params(0)
    sizes = [(27 * 8 * 32, 32), (27 * 32 * 32, 32), (27 * 32 * 8, 8)]
    assert p.dtype == np.float32 and p.size == sum(w + b for w, b in sizes)
    off = 0
    for (nw, nb), cin in zip(sizes, (8, 32, 32)):
        w, b = p[off:off + nw], p[off + nw:off + nw + nb]
        off += nw + nb
        assert np.all(b == 0.0)
        std = np.sqrt(2.0 / (27 * cin)) * (0.01 if nb == 8 else 1.0)
        assert np.std(w) == pytest.approx(std, rel=0.1)
    assert np.array_equal(CT.init_params(0), p) and not np.array_equal(CT.init_params(1), p)
