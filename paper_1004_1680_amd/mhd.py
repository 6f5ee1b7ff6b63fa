"""Python binding of the HIP MHD library (``libmhd.so``, C ABI in include/mhd.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  If the library is missing this module raises on
import of the library (``load()``); there is no CPU fallback.

The functions ``mhd_*`` mirror the C ABI one to one.  ``Solver`` wraps a
handle for numpy host arrays of shape ``(8, nz, ny, nx)`` (float64) and for
torch device tensors (PyTorch is used only for device memory and streams).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhd.so")

MHD_OK, MHD_EINVAL, MHD_ENOMEM, MHD_EDEVICE, MHD_ENONPHYS, MHD_ESTATE = 0, -1, -2, -3, -4, -5
MHD_F32, MHD_F64 = 0, 1
MHD_TUNE_CHUNK_Y, MHD_TUNE_CHUNK_Z, MHD_TUNE_REVERSE = 1, 2, 3
MHD_TUNE_PAIR_CHUNK_Y, MHD_TUNE_PAIR_CHUNK_Z, MHD_TUNE_WIDE_OFFSETS = 4, 5, 6
MHD_TUNE_MIDDLE, MHD_TUNE_MIDDLE_CHUNK, MHD_TUNE_ROW_GROUP = 7, 8, 9
MHD_BATCH_GRID_X, MHD_BATCH_GRID_Y, MHD_BATCH_GRID_Z, MHD_BATCH_CHUNK = 10, 11, 12, 13
MHD_BATCH_REVERSE, MHD_BATCH_WIDE_OFFSETS, MHD_BATCH_PAIR_CHUNK, MHD_BATCH_MIDDLE = 14, 15, 16, 17
MHD_LIMITER_VANLEER, MHD_LIMITER_MINMOD, MHD_LIMITER_MC, MHD_LIMITER_SUPERBEE = 0, 1, 2, 3
MHD_FREEZE_STEP, MHD_FREEZE_CELL, MHD_FREEZE_PENCIL = 0, 1, 2

_lib = None


class MHDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class NonPhysicalState(MHDError):
    pass


def load():
    """Load libmhd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} not built: run python -m paper_1004_1680_amd.build")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7.
    # Loading torch first makes the dynamic loader bind libmhd.so to that
    # same runtime (same soname), so torch's streams and device pointers are
    # native to the library; the other order would bring up a second runtime
    # that keeps torch from seeing the GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    fp = ctypes.POINTER(ctypes.c_float)
    sig = {
        "mhd_create": (vp, [i, i, i, d]),
        "mhd_create_ex": (vp, [i, i, i, d, i, vp, vp, vp]),
        "mhd_destroy": (None, [vp]),
        "mhd_info": (i, [vp, ip, ip]),
        "mhd_set_state": (i, [vp, dp, sz]),
        "mhd_get_state": (i, [vp, dp, sz]),
        "mhd_set_state_device": (i, [vp, vp, sz, i]),
        "mhd_get_state_device": (i, [vp, vp, sz, i]),
        "mhd_cfl_dt": (i, [vp, d, dp]),
        "mhd_set_relaxation_speed": (i, [vp, d]),
        "mhd_get_relaxation_speed": (i, [vp, dp]),
        "mhd_fluid": (i, [vp, i, d]),
        "mhd_magnetic": (i, [vp, i, d]),
        "mhd_sweep": (i, [vp, i, d]),
        "mhd_step": (i, [vp, d]),
        "mhd_step_auto": (i, [vp, d]),
        "mhd_status": (i, [vp, ctypes.POINTER(ctypes.c_longlong)]),
        "mhd_time": (i, [vp, dp]),
        "mhd_diag": (i, [vp, dp]),
        "mhd_restrict": (i, [vp, vp]),
        "mhd_set_launch": (i, [vp, i, i]),
        "mhd_get_launch": (i, [vp, i, ip]),
        "mhd_set_limiter": (i, [vp, i]),
        "mhd_get_limiter": (i, [vp, ip]),
        "mhd_set_freezing_speed": (i, [vp, i]),
        "mhd_get_freezing_speed": (i, [vp, ip]),
        "mhd_batch_create": (vp, [i, ip, d, i, vp]),
        "mhd_batch_destroy": (None, [vp]),
        "mhd_batch_info": (i, [vp, ip, ctypes.POINTER(ctypes.c_longlong)]),
        "mhd_batch_set_state": (i, [vp, i, dp, sz]),
        "mhd_batch_get_state": (i, [vp, i, dp, sz]),
        "mhd_batch_step_auto": (i, [vp, d]),
        "mhd_batch_run": (i, [vp, d, i, i]),
        "mhd_batch_status": (i, [vp, ctypes.POINTER(ctypes.c_longlong), ip]),
        "mhd_batch_time": (i, [vp, dp]),
        "mhd_batch_set_launch": (i, [vp, i, i]),
        "mhd_batch_get_launch": (i, [vp, i, ip]),
        "mhd_batch_set_limiter": (i, [vp, i]),
        "mhd_batch_get_limiter": (i, [vp, ip]),
        "mhd_closure_create": (vp, [i, i, i, vp]),
        "mhd_closure_destroy": (None, [vp]),
        "mhd_closure_set_params": (i, [vp, fp, sz]),
        "mhd_closure_get_params": (i, [vp, fp, sz]),
        "mhd_closure_set_scales": (i, [vp, fp, fp, fp, fp]),
        "mhd_closure_forward": (i, [vp, vp, vp]),
        "mhd_closure_grad": (i, [vp, vp, vp, dp, fp, sz]),
        "mhd_closure_train_step": (i, [vp, vp, vp, ctypes.c_float, dp]),
        "mhd_closure_step": (i, [vp, vp, d]),
        "mhd_closure_fallbacks": (i, [vp, ip]),
        "mhd_closure_reduced": (i, [vp, ip]),
        "mhd_closure_residual": (i, [vp, vp, vp, vp]),
        "mhd_closure_stats": (i, [vp, vp, vp, dp]),
        "mhd_closure_set_gate": (i, [vp, fp]),
        "mhd_closure_get_gate": (i, [vp, vp]),
        "mhd_conv3d_forward": (i, [ip, i, i, vp, fp, fp, vp, vp]),
        "mhd_conv3d_dgrad": (i, [ip, i, i, vp, fp, vp, vp]),
        "mhd_conv3d_wgrad": (i, [ip, i, i, vp, vp, fp, fp, vp]),
        "mhd_stream_copy": (i, [vp, vp, sz, vp]),
        "mhd_cfl_dt_noalloc": (i, [vp, i, i, i, i, d, d, vp, vp]),
        "mhd_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return [l for l in ("mhd_create", "mhd_create_ex", "mhd_destroy", "mhd_info", "mhd_set_state",
                        "mhd_get_state", "mhd_set_state_device", "mhd_get_state_device",
                        "mhd_cfl_dt", "mhd_set_relaxation_speed", "mhd_get_relaxation_speed",
                        "mhd_fluid", "mhd_magnetic", "mhd_sweep", "mhd_step", "mhd_step_auto",
                        "mhd_status", "mhd_time", "mhd_diag", "mhd_restrict", "mhd_set_launch",
                        "mhd_get_launch", "mhd_set_limiter", "mhd_get_limiter", "mhd_set_freezing_speed",
                        "mhd_get_freezing_speed", "mhd_batch_create", "mhd_batch_destroy",
                        "mhd_batch_info", "mhd_batch_set_state", "mhd_batch_get_state",
                        "mhd_batch_step_auto", "mhd_batch_run", "mhd_batch_status",
                        "mhd_batch_time", "mhd_batch_set_launch", "mhd_batch_get_launch",
                        "mhd_batch_set_limiter", "mhd_batch_get_limiter",
                        "mhd_closure_create", "mhd_closure_destroy", "mhd_closure_set_params",
                        "mhd_closure_get_params", "mhd_closure_set_scales", "mhd_closure_forward",
                        "mhd_closure_grad", "mhd_closure_train_step", "mhd_closure_step",
                        "mhd_closure_fallbacks", "mhd_closure_reduced", "mhd_closure_residual", "mhd_closure_stats",
                        "mhd_closure_set_gate", "mhd_closure_get_gate",
                        "mhd_conv3d_forward", "mhd_conv3d_dgrad",
                        "mhd_conv3d_wgrad", "mhd_stream_copy", "mhd_cfl_dt_noalloc",
                        "mhd_last_error")]


def last_error():
    return load().mhd_last_error().decode()


def check(r):
    if r != MHD_OK:
        msg = last_error()
        if r == MHD_ENONPHYS:
            raise NonPhysicalState(r, msg)
        raise MHDError(r, msg)
    return r


# --- one-to-one wrappers of the C ABI ---------------------------------------

def mhd_create(nx, ny, nz, gamma):
    return load().mhd_create(nx, ny, nz, gamma)


def mhd_create_ex(nx, ny, nz, gamma, prec, stream=None, dev_buf_a=None, dev_buf_b=None):
    return load().mhd_create_ex(nx, ny, nz, gamma, prec, stream, dev_buf_a, dev_buf_b)


def mhd_destroy(h):
    load().mhd_destroy(h)


def mhd_set_state(h, host):
    host = np.ascontiguousarray(host, dtype=np.float64)
    return load().mhd_set_state(h, host.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), host.size)


def mhd_get_state(h, out):
    return load().mhd_get_state(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size)


def mhd_cfl_dt(h, cfl):
    dt = ctypes.c_double(0.0)
    r = load().mhd_cfl_dt(h, cfl, ctypes.byref(dt))
    return r, dt.value


def mhd_fluid(h, dim, dt):
    return load().mhd_fluid(h, dim, dt)


def mhd_magnetic(h, dim, dt):
    return load().mhd_magnetic(h, dim, dt)


def mhd_sweep(h, dim, dt):
    return load().mhd_sweep(h, dim, dt)


def mhd_step(h, dt):
    return load().mhd_step(h, dt)


def mhd_step_auto(h, cfl):
    return load().mhd_step_auto(h, cfl)


def mhd_diag(h):
    out = (ctypes.c_double * 9)()
    r = load().mhd_diag(h, out)
    return r, np.array(out[:])


def mhd_restrict(fine, coarse):
    return load().mhd_restrict(fine, coarse)


# --- convenience handle ------------------------------------------------------

def _torch_stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Solver:
    """One periodic grid of n = (nx, ny, nz) cells on the current HIP device.

    prec: "f32" or "f64".  stream: a torch.cuda.Stream (or raw handle) on
    which every kernel is enqueued; None = the default stream.  buffers: None
    (the library allocates the two state buffers) or two contiguous device
    tensors of the tier's dtype with at least 8*nx*ny*nz elements each; the
    Solver keeps references to them until it is closed."""

    def __init__(self, n, gamma=5.0 / 3.0, prec="f32", stream=None, buffers=None):
        self.lib = load()
        self.n = tuple(int(v) for v in n)
        self.gamma = float(gamma)
        self.prec = {"f32": MHD_F32, "f64": MHD_F64}[prec]
        self._buffers = None
        ptrs = (None, None)
        if buffers is not None:
            import torch
            a, b = buffers
            want = torch.float64 if self.prec == MHD_F64 else torch.float32
            need = 8 * self.n[0] * self.n[1] * self.n[2]
            for t in (a, b):
                if not (t.is_cuda and t.is_contiguous() and t.dtype == want and t.numel() >= need):
                    raise ValueError(f"state buffers: contiguous {want} device tensors of at least "
                                     f"{need} elements")
            self._buffers = (a, b)
            ptrs = (a.data_ptr(), b.data_ptr())
        self.h = self.lib.mhd_create_ex(self.n[0], self.n[1], self.n[2], self.gamma, self.prec,
                                        _torch_stream(stream), *ptrs)
        if not self.h:
            self._buffers = None
            raise MHDError(MHD_EINVAL, last_error())

    def close(self):
        if self.h:
            self.lib.mhd_destroy(self.h)
            self.h = None
        self._buffers = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (8, self.n[2], self.n[1], self.n[0])

    @property
    def ncell(self):
        return self.n[0] * self.n[1] * self.n[2]

    def set_state(self, s):
        s = np.ascontiguousarray(s, dtype=np.float64)
        if s.shape != self.shape:
            raise ValueError(f"state shape {s.shape} != {self.shape}")
        check(self.lib.mhd_set_state(self.h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     s.size))

    def get_state(self):
        out = np.empty(self.shape, dtype=np.float64)
        check(self.lib.mhd_get_state(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     out.size))
        return out

    def set_state_tensor(self, t):
        """t: contiguous torch CUDA tensor (float32 or float64) of shape self.shape"""
        import torch
        prec = MHD_F64 if t.dtype == torch.float64 else MHD_F32
        assert t.is_cuda and t.is_contiguous() and tuple(t.shape) == self.shape
        check(self.lib.mhd_set_state_device(self.h, ctypes.c_void_p(t.data_ptr()), t.numel(), prec))

    def get_state_tensor(self, out=None, dtype=None):
        import torch
        if out is None:
            dtype = dtype or (torch.float64 if self.prec == MHD_F64 else torch.float32)
            out = torch.empty(self.shape, dtype=dtype, device="cuda")
        prec = MHD_F64 if out.dtype == torch.float64 else MHD_F32
        check(self.lib.mhd_get_state_device(self.h, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                            prec))
        return out

    def cfl_dt(self, cfl=0.7):
        dt = ctypes.c_double(0.0)
        check(self.lib.mhd_cfl_dt(self.h, cfl, ctypes.byref(dt)))
        return dt.value

    def set_relaxation_speed(self, c):
        check(self.lib.mhd_set_relaxation_speed(self.h, c))

    def relaxation_speed(self):
        c = ctypes.c_double(0.0)
        check(self.lib.mhd_get_relaxation_speed(self.h, ctypes.byref(c)))
        return c.value

    def fluid(self, dim, dt):
        check(self.lib.mhd_fluid(self.h, dim, dt))

    def magnetic(self, dim, dt):
        check(self.lib.mhd_magnetic(self.h, dim, dt))

    def sweep(self, code, dt):
        check(self.lib.mhd_sweep(self.h, code, dt))

    def step(self, dt):
        check(self.lib.mhd_step(self.h, dt))

    def step_auto(self, cfl=0.7):
        check(self.lib.mhd_step_auto(self.h, cfl))

    def status(self):
        n = ctypes.c_longlong(0)
        check(self.lib.mhd_status(self.h, ctypes.byref(n)))
        return n.value

    def time(self):
        t = ctypes.c_double(0.0)
        check(self.lib.mhd_time(self.h, ctypes.byref(t)))
        return t.value

    def diag(self):
        out = (ctypes.c_double * 9)()
        check(self.lib.mhd_diag(self.h, out))
        return np.array(out[:])

    def set_chunk(self, axis, value):
        """march chunk length along axis 1 (y) or 2 (z); 0 = built-in"""
        check(self.lib.mhd_set_launch(self.h, axis, value))

    def chunk(self, axis):
        v = ctypes.c_int(0)
        check(self.lib.mhd_get_launch(self.h, axis, ctypes.byref(v)))
        return v.value

    def set_launch(self, key, value):
        """any MHD_TUNE_* launch-shape key (results do not depend on them)"""
        check(self.lib.mhd_set_launch(self.h, key, value))

    def launch(self, key):
        v = ctypes.c_int(0)
        check(self.lib.mhd_get_launch(self.h, key, ctypes.byref(v)))
        return v.value

    def set_pair_chunk(self, axis, value):
        """march chunk of the fused reverse-half pair along axis 1 (y) or 2
        (z); 0 = built-in"""
        check(self.lib.mhd_set_launch(self.h, MHD_TUNE_PAIR_CHUNK_Y + axis - 1, value))

    def pair_chunk(self, axis):
        v = ctypes.c_int(0)
        check(self.lib.mhd_get_launch(self.h, MHD_TUNE_PAIR_CHUNK_Y + axis - 1, ctypes.byref(v)))
        return v.value

    def set_reverse(self, value):
        """reverse-half pairs M_d F_d: 1 one fused launch each, 2 the two
        operators in turn, 0 built-in (same results either way)"""
        check(self.lib.mhd_set_launch(self.h, MHD_TUNE_REVERSE, value))

    def reverse(self):
        v = ctypes.c_int(0)
        check(self.lib.mhd_get_launch(self.h, MHD_TUNE_REVERSE, ctypes.byref(v)))
        return v.value

    def set_limiter(self, kind):
        """slope limiter of the operators: MHD_LIMITER_VANLEER (the paper's,
        default), _MINMOD, _MC or _SUPERBEE; other than van Leer's, the
        reverse pairs run as two launches each"""
        check(self.lib.mhd_set_limiter(self.h, kind))

    def limiter(self):
        v = ctypes.c_int(0)
        check(self.lib.mhd_get_limiter(self.h, ctypes.byref(v)))
        return v.value

    def set_freezing(self, mode):
        """freezing speed of the fluid operator: MHD_FREEZE_STEP (one number
        per step, default), MHD_FREEZE_CELL or MHD_FREEZE_PENCIL (method
        variants, van Leer's limiter only)"""
        check(self.lib.mhd_set_freezing_speed(self.h, mode))

    def freezing(self):
        v = ctypes.c_int(0)
        check(self.lib.mhd_get_freezing_speed(self.h, ctypes.byref(v)))
        return v.value

    def restrict_to(self, coarse):
        check(self.lib.mhd_restrict(self.h, coarse.h))

    def run(self, nsteps, cfl=0.7, t_end=None):
        """nsteps full steps, dt from the CFL condition before each (host
        path).  With t_end, the last step is shortened to end exactly there.
        Returns the list of dt."""
        dts = []
        t = 0.0
        for _ in range(nsteps if t_end is None else 10 ** 9):
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            dt = self.cfl_dt(cfl)
            if t_end is not None:
                dt = min(dt, 0.5 * (t_end - t))
            self.step(dt)
            t += 2.0 * dt
            dts.append(dt)
        return dts


class Batch:
    """Ensemble of independent periodic boxes advanced together: one
    persistent launch per operator over all boxes, per-box CFL time step,
    optional HIP-graph replay of the step.  dims: list of (nx, ny, nz)."""

    def __init__(self, dims, gamma=5.0 / 3.0, prec="f32", stream=None):
        self.lib = load()
        self.dims = [tuple(int(v) for v in n) for n in dims]
        self.nbox = len(self.dims)
        self.prec = {"f32": MHD_F32, "f64": MHD_F64}[prec]
        arr = (ctypes.c_int * (3 * self.nbox))(*[v for n in self.dims for v in n])
        self.h = self.lib.mhd_batch_create(self.nbox, arr, float(gamma), self.prec,
                                           _torch_stream(stream))
        if not self.h:
            raise MHDError(MHD_EINVAL, last_error())

    def close(self):
        if self.h:
            self.lib.mhd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncell(self):
        return sum(n[0] * n[1] * n[2] for n in self.dims)

    def shape(self, box):
        n = self.dims[box]
        return (8, n[2], n[1], n[0])

    def set_state(self, box, s):
        s = np.ascontiguousarray(s, dtype=np.float64)
        if s.shape != self.shape(box):
            raise ValueError(f"state shape {s.shape} != {self.shape(box)}")
        check(self.lib.mhd_batch_set_state(self.h, box,
                                           s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), s.size))

    def get_state(self, box):
        out = np.empty(self.shape(box), dtype=np.float64)
        check(self.lib.mhd_batch_get_state(self.h, box,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
        return out

    def step_auto(self, cfl=0.7):
        check(self.lib.mhd_batch_step_auto(self.h, cfl))

    def run(self, nsteps, cfl=0.7, graph=True):
        check(self.lib.mhd_batch_run(self.h, cfl, nsteps, 1 if graph else 0))

    def status(self, raise_on_nonphysical=True):
        steps = (ctypes.c_longlong * self.nbox)()
        nonphys = (ctypes.c_int * self.nbox)()
        r = self.lib.mhd_batch_status(self.h, steps, nonphys)
        if r != MHD_ENONPHYS or raise_on_nonphysical:
            check(r)
        return np.array(steps[:]), np.array(nonphys[:])

    def times(self):
        t = (ctypes.c_double * self.nbox)()
        check(self.lib.mhd_batch_time(self.h, t))
        return np.array(t[:])

    def set_launch(self, key, value):
        check(self.lib.mhd_batch_set_launch(self.h, key, value))

    def launch(self, key):
        v = ctypes.c_int(0)
        check(self.lib.mhd_batch_get_launch(self.h, key, ctypes.byref(v)))
        return v.value

    def set_limiter(self, kind):
        """slope limiter of every box (MHD_LIMITER_*; van Leer's by default)"""
        check(self.lib.mhd_batch_set_limiter(self.h, kind))

    def limiter(self):
        v = ctypes.c_int(0)
        check(self.lib.mhd_batch_get_limiter(self.h, ctypes.byref(v)))
        return v.value


# --- learned closure ---------------------------------------------------------

NPARAM = 27 * 8 * 32 + 32 + 27 * 32 * 32 + 32 + 27 * 32 * 8 + 8


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Closure:
    """Learned correction of a coarse grid n (multiples of 32).  Device
    arrays are torch CUDA float32 tensors of shape (8, nz, ny, nx)."""

    def __init__(self, n, stream=None):
        self.lib = load()
        self.n = tuple(int(v) for v in n)
        self.stream = stream
        self.h = self.lib.mhd_closure_create(self.n[0], self.n[1], self.n[2], _torch_stream(stream))
        if not self.h:
            raise MHDError(MHD_EINVAL, last_error())

    def close(self):
        if self.h:
            self.lib.mhd_closure_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        check(self.lib.mhd_closure_set_params(self.h, _fptr(p), p.size))

    def params(self):
        p = np.empty(NPARAM, dtype=np.float32)
        check(self.lib.mhd_closure_get_params(self.h, _fptr(p), p.size))
        return p

    def set_scales(self, in_mean, in_std, out_scale, target_scale):
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (in_mean, in_std, out_scale, target_scale)]
        check(self.lib.mhd_closure_set_scales(self.h, *[_fptr(v) for v in a]))

    def forward(self, u, out=None):
        import torch
        out = torch.empty_like(u) if out is None else out
        check(self.lib.mhd_closure_forward(self.h, _dptr(u), _dptr(out)))
        return out

    def grad(self, u, target):
        g = np.empty(NPARAM, dtype=np.float32)
        L = ctypes.c_double(0.0)
        check(self.lib.mhd_closure_grad(self.h, _dptr(u), _dptr(target), ctypes.byref(L), _fptr(g), g.size))
        return L.value, g

    def train_step(self, u, target, lr, want_loss=True):
        L = ctypes.c_double(0.0)
        check(self.lib.mhd_closure_train_step(self.h, _dptr(u), _dptr(target), ctypes.c_float(lr),
                                              ctypes.byref(L) if want_loss else None))
        return L.value if want_loss else None

    def step(self, solver, cfl=0.7):
        check(self.lib.mhd_closure_step(self.h, solver.h, cfl))

    def fallbacks(self):
        v = ctypes.c_int(0)
        check(self.lib.mhd_closure_fallbacks(self.h, ctypes.byref(v)))
        return v.value

    def reduced(self):
        """learned steps whose correction was applied with theta < 1"""
        v = ctypes.c_int(0)
        check(self.lib.mhd_closure_reduced(self.h, ctypes.byref(v)))
        return v.value

    def residual(self, u_ref, u_plain, out=None):
        """target = u_ref - u_plain (device tensors, computed by the library)"""
        import torch
        out = torch.empty_like(u_plain) if out is None else out
        check(self.lib.mhd_closure_residual(self.h, _dptr(u_ref), _dptr(u_plain), _dptr(out)))
        return out

    def stats(self, u, target):
        """FP64 per-field sums: rows sum u, sum u^2, sum |u|, sum |target|,
        sum of the roughness of u"""
        out = (ctypes.c_double * 40)()
        check(self.lib.mhd_closure_stats(self.h, _dptr(u), _dptr(target), out))
        return np.array(out[:]).reshape(5, 8)

    def set_gate(self, mean_roughness):
        """roughness gate with the training-set mean roughness per field
        (None: no gate)"""
        if mean_roughness is None:
            check(self.lib.mhd_closure_set_gate(self.h, None))
            return
        r = np.ascontiguousarray(mean_roughness, dtype=np.float32)
        check(self.lib.mhd_closure_set_gate(self.h, _fptr(r)))

    def gate(self):
        """gate of the last forward pass (torch CUDA tensor of nx*ny*nz)"""
        import torch
        out = torch.empty(self.n[0] * self.n[1] * self.n[2], dtype=torch.float32, device="cuda")
        check(self.lib.mhd_closure_get_gate(self.h, _dptr(out)))
        return out


def conv3d_forward(n, x, w, bias, y, stream=None):
    """x: bf16 bits (torch int16/uint16 CUDA) [cell][cin]; w numpy [27][cin][cout];
    y: torch float32 CUDA [cell][cout]"""
    w = np.ascontiguousarray(w, dtype=np.float32)
    b = None if bias is None else np.ascontiguousarray(bias, dtype=np.float32)
    nn = (ctypes.c_int * 3)(*n)
    check(load().mhd_conv3d_forward(nn, w.shape[1], w.shape[2], _dptr(x), _fptr(w),
                                    _fptr(b) if b is not None else None, _dptr(y), _torch_stream(stream)))


def conv3d_dgrad(n, dy, w, dx, stream=None):
    w = np.ascontiguousarray(w, dtype=np.float32)
    nn = (ctypes.c_int * 3)(*n)
    check(load().mhd_conv3d_dgrad(nn, w.shape[1], w.shape[2], _dptr(dy), _fptr(w), _dptr(dx),
                                  _torch_stream(stream)))


def conv3d_wgrad(n, cin, cout, xT, dyT, stream=None):
    dw = np.empty((27, cin, cout), dtype=np.float32)
    db = np.empty(cout, dtype=np.float32)
    nn = (ctypes.c_int * 3)(*n)
    check(load().mhd_conv3d_wgrad(nn, cin, cout, _dptr(xT), _dptr(dyT), _fptr(dw), _fptr(db),
                                  _torch_stream(stream)))
    return dw, db


def stream_copy(src, dst, stream=None):
    """plain device copy of a tensor's bytes into another of the same size
    (the streaming-bandwidth reference); asynchronous on `stream`"""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("source and destination sizes differ")
    check(load().mhd_stream_copy(_dptr(src), _dptr(dst), nbytes, _torch_stream(stream)))


def cfl_dt_noalloc(state, n, gamma=5.0 / 3.0, cfl=0.7, out=None, stream=None):
    """mhd_cfl_dt_noalloc on a device tensor `state` (8 * nx*ny*nz float32 or
    float64 values, state layout) of grid n = (nx, ny, nz): enqueues the CFL
    reduction (no allocation) writing (dt, vmax, record) into the float64
    device tensor `out` (3 values; created if None) and returns it"""
    import torch
    if state.dtype == torch.float32:
        prec = MHD_F32
    elif state.dtype == torch.float64:
        prec = MHD_F64
    else:
        raise ValueError("state must be float32 or float64")
    if state.numel() != 8 * n[0] * n[1] * n[2] or not state.is_contiguous():
        raise ValueError("state must be a contiguous tensor of 8 * nx * ny * nz values")
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=state.device)
    check(load().mhd_cfl_dt_noalloc(_dptr(state), int(n[0]), int(n[1]), int(n[2]), prec, float(gamma),
                                    float(cfl), _dptr(out), _torch_stream(stream)))
    return out
