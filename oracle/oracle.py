"""ctypes wrapper of the FP64 C oracle (test infrastructure only).

The oracle implements the ideal-MHD update step of Pang, Pen & Perrone
(arXiv:1004.1680), section II, as plain whole-array loops in C, compiled with
gcc and ``-ffp-contract=off``.  States are numpy float64 arrays of shape
``(8, nz, ny, nx)``: rho, m_x, m_y, m_z, e, b_x, b_y, b_z (b on low faces).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhd_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "closure_oracle.c")]
_LIB = os.path.join(_HERE, "libmhd_oracle.so")
_lib = None

__all__ = ["build", "load", "fluid_sweep", "mag_sweep", "sweep", "step",
           "cfl", "cfl_dt", "diag", "restrict", "run", "NonPhysical",
           "limiter_value", "VANLEER", "MINMOD", "MC", "SUPERBEE",
           "FREEZE_GRID", "FREEZE_CELL", "FREEZE_PENCIL"]


class NonPhysical(RuntimeError):
    pass


def build(verbose=False):
    """Compile the oracle with gcc (no fused multiply-add, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", _LIB, *_SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(p) for p in _SRCS):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i, d = ctypes.c_int, ctypes.c_double
    lib.oracle_fluid_sweep.argtypes = [i, i, i, d, dp, dp, i, d, d]
    lib.oracle_mag_sweep.argtypes = [i, i, i, d, dp, dp, i, d]
    lib.oracle_sweep.argtypes = [i, i, i, d, dp, i, d, d]
    lib.oracle_step.argtypes = [i, i, i, d, dp, d, d]
    lib.oracle_cfl.argtypes = [i, i, i, d, dp, d, dp, dp]
    lib.oracle_diag.argtypes = [i, i, i, dp, dp]
    lib.oracle_diag.restype = None
    lib.oracle_restrict.argtypes = [i, i, i, i, dp, dp]
    lib.oracle_conv3d.argtypes = [i, i, i, i, i, dp, dp, dp, dp]
    lib.oracle_conv3d_dgrad.argtypes = [i, i, i, i, i, dp, dp, dp]
    lib.oracle_conv3d_wgrad.argtypes = [i, i, i, i, i, dp, dp, dp, dp]
    lib.oracle_closure_project.argtypes = [i, i, i, dp, dp, dp]
    lib.oracle_closure_project_T.argtypes = [i, i, i, dp, dp, dp]
    lib.oracle_closure_gate.argtypes = [i, i, i, dp, dp, dp]
    for fn in ("oracle_conv3d", "oracle_conv3d_dgrad", "oracle_conv3d_wgrad",
               "oracle_closure_project", "oracle_closure_project_T", "oracle_closure_gate"):
        getattr(lib, fn).restype = None
    lib.oracle_set_limiter.argtypes = [i]
    lib.oracle_set_freeze.argtypes = [i]
    lib.oracle_limiter_value.argtypes = [i, d, d]
    lib.oracle_limiter_value.restype = d
    for fn in ("oracle_fluid_sweep", "oracle_mag_sweep", "oracle_sweep",
               "oracle_step", "oracle_cfl", "oracle_restrict", "oracle_set_limiter",
               "oracle_set_freeze"):
        getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(s):
    s = np.ascontiguousarray(s, dtype=np.float64)
    assert s.ndim == 4 and s.shape[0] == 8, s.shape
    return s


def _dims(s):
    return s.shape[3], s.shape[2], s.shape[1]


# slope limiters: 0 van Leer (section II.B), 1 minmod, 2 MC, 3 superbee
VANLEER, MINMOD, MC, SUPERBEE = 0, 1, 2, 3


# freezing (relaxation) speed of the fluid sweeps: 0 one number per step
# (the c argument; the reading taken for the paper's method), 1 |v_n| +
# c_fast per cell, 2 its largest value along the pencil (method variants)
FREEZE_GRID, FREEZE_CELL, FREEZE_PENCIL = 0, 1, 2


class _Limiter:
    """the oracle's process-wide limiter and freezing-speed mode for the
    duration of one call"""

    def __init__(self, kind, freeze=FREEZE_GRID):
        self.kind = kind
        self.freeze = freeze

    def __enter__(self):
        if load().oracle_set_limiter(self.kind) != 0:
            raise ValueError(f"unknown limiter {self.kind}")
        if load().oracle_set_freeze(self.freeze) != 0:
            load().oracle_set_limiter(VANLEER)
            raise ValueError(f"unknown freezing-speed mode {self.freeze}")

    def __exit__(self, *exc):
        load().oracle_set_limiter(VANLEER)
        load().oracle_set_freeze(FREEZE_GRID)


def limiter_value(kind, a, b):
    """phi(a, b) of the limiter `kind` on two halved one-sided differences"""
    return load().oracle_limiter_value(kind, a, b)


def fluid_sweep(s, d, dt, c, gamma=5.0 / 3.0, limiter=VANLEER, freeze=FREEZE_GRID):
    """Fluid operator along axis d with relaxation speed c (freeze: see
    FREEZE_*; c is unused by the per-cell and per-pencil variants)."""
    s = _check(s)
    out = np.empty_like(s)
    nx, ny, nz = _dims(s)
    with _Limiter(limiter, freeze):
        r = load().oracle_fluid_sweep(nx, ny, nz, gamma, _ptr(s), _ptr(out), d, dt, c)
    assert r == 0
    return out


def mag_sweep(s, d, dt, gamma=5.0 / 3.0, limiter=VANLEER):
    """Magnetic advection-constraint operator along axis d."""
    s = _check(s)
    out = np.empty_like(s)
    nx, ny, nz = _dims(s)
    with _Limiter(limiter):
        r = load().oracle_mag_sweep(nx, ny, nz, gamma, _ptr(s), _ptr(out), d, dt)
    assert r == 0
    return out


def sweep(s, code, dt, c, gamma=5.0 / 3.0, limiter=VANLEER, freeze=FREEZE_GRID):
    """code 0..2: fluid then magnetic along code; 3..5: the reverse along
    code-3."""
    s = _check(s).copy()
    nx, ny, nz = _dims(s)
    with _Limiter(limiter, freeze):
        assert load().oracle_sweep(nx, ny, nz, gamma, _ptr(s), code, dt, c) == 0
    return s


def step(s, dt, c, gamma=5.0 / 3.0, limiter=VANLEER, freeze=FREEZE_GRID):
    """Full Strang step (x, y, z, z, y, x) of 2 dt with relaxation speed c."""
    s = _check(s).copy()
    nx, ny, nz = _dims(s)
    with _Limiter(limiter, freeze):
        assert load().oracle_step(nx, ny, nz, gamma, _ptr(s), dt, c) == 0
    return s


def cfl(s, cfl=0.7, gamma=5.0 / 3.0):
    """(dt, vmax): CFL time step and the largest signal speed."""
    s = _check(s)
    nx, ny, nz = _dims(s)
    dt = ctypes.c_double(0.0)
    vm = ctypes.c_double(0.0)
    r = load().oracle_cfl(nx, ny, nz, gamma, _ptr(s), cfl, ctypes.byref(dt),
                          ctypes.byref(vm))
    if r == -4:
        raise NonPhysical("non-physical state (rho<=0, p<0 or non-finite)")
    assert r == 0, r
    return dt.value, vm.value


def cfl_dt(s, cfl_number=0.7, gamma=5.0 / 3.0):
    return cfl(s, cfl_number, gamma)[0]


def diag(s):
    s = _check(s)
    nx, ny, nz = _dims(s)
    out = np.zeros(9)
    load().oracle_diag(nx, ny, nz, _ptr(s), _ptr(out))
    return out


def restrict(s, r):
    s = _check(s)
    nx, ny, nz = _dims(s)
    out = np.zeros((8, nz // r, ny // r, nx // r))
    assert load().oracle_restrict(nx, ny, nz, r, _ptr(s), _ptr(out)) == 0
    return out


def run(s, nsteps, cfl_number=0.7, gamma=5.0 / 3.0, t_end=None, limiter=VANLEER,
        freeze=FREEZE_GRID):
    """Advance nsteps full steps with dt from the CFL condition before each
    step.  If t_end is given, stop there, shortening the last step so that
    the run ends exactly at t_end.  Returns (state, time, list of dt)."""
    s = _check(s).copy()
    t = 0.0
    dts = []
    for _ in range(nsteps if t_end is None else 10 ** 9):
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        dt, vmax = cfl(s, cfl_number, gamma)
        if t_end is not None:
            dt = min(dt, 0.5 * (t_end - t))
        s = step(s, dt, vmax, gamma, limiter, freeze)
        t += 2.0 * dt
        dts.append(dt)
    return s, t, dts
