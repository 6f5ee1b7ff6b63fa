"""The C-ABI library loads and exports every symbol include/mhd.h declares,
and rejects bad arguments before touching a device (no compute on CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "mhd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("mhd_create", "mhd_set_state", "mhd_cfl_dt", "mhd_sweep", "mhd_step",
                 "mhd_get_state", "mhd_restrict", "mhd_diag"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1004_1680_amd import mhd
    lib = mhd.load()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps each of them under the same name
    assert sorted(mhd.exported_symbols()) == declared_symbols()


@pytest.mark.parametrize("dims", [(7, 8, 8), (8, 6, 8), (8, 8, 10), (0, 8, 8), (8, 8, 4)])
def test_bad_dimensions_rejected(dims):
    from paper_1004_1680_amd import mhd
    lib = mhd.load()
    assert not lib.mhd_create(*dims, 5.0 / 3.0)
    assert "grid dimension" in mhd.last_error()


@pytest.mark.parametrize("gamma", [1.0, 0.5, float("nan")])
def test_bad_gamma_rejected(gamma):
    from paper_1004_1680_amd import mhd
    assert not mhd.load().mhd_create(8, 8, 8, gamma)
    assert "gamma" in mhd.last_error()


def test_bad_precision_rejected():
    from paper_1004_1680_amd import mhd
    assert not mhd.load().mhd_create_ex(8, 8, 8, 5.0 / 3.0, 7, None, None, None)
    assert "precision" in mhd.last_error()


def test_one_state_buffer_rejected():
    from paper_1004_1680_amd import mhd
    lib = mhd.load()
    assert not lib.mhd_create_ex(8, 8, 8, 5.0 / 3.0, 0, None, 1 << 20, None)
    assert "both state buffers" in mhd.last_error()
    assert not lib.mhd_create_ex(8, 8, 8, 5.0 / 3.0, 0, None, None, 1 << 20)
    assert "both state buffers" in mhd.last_error()


def test_null_handle_calls_fail_cleanly():
    from paper_1004_1680_amd import mhd
    lib = mhd.load()
    assert lib.mhd_step(None, 0.1) == mhd.MHD_EINVAL
    assert lib.mhd_sweep(None, 7, 0.1) == mhd.MHD_EINVAL
    assert lib.mhd_fluid(None, 3, 0.1) == mhd.MHD_EINVAL
    assert lib.mhd_diag(None, None) == mhd.MHD_EINVAL
    lib.mhd_destroy(None)


def test_library_shares_torchs_hip_runtime():
    """after load(), exactly one libamdhip64 is mapped in the process: the
    one torch loaded (two HIP runtimes in one process keep torch from seeing
    the GPU once the library's runtime initialised first)"""
    from paper_1004_1680_amd import mhd
    mhd.load()
    with open("/proc/self/maps") as f:
        libs = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(libs) == 1, libs


def test_limiter_calls_on_a_null_handle_fail_cleanly():
    import ctypes
    from paper_1004_1680_amd import mhd
    lib = mhd.load()
    assert lib.mhd_set_limiter(None, 1) == mhd.MHD_EINVAL
    v = ctypes.c_int(7)
    assert lib.mhd_get_limiter(None, ctypes.byref(v)) == mhd.MHD_EINVAL
    assert lib.mhd_batch_set_limiter(None, 1) == mhd.MHD_EINVAL
    assert lib.mhd_batch_get_limiter(None, ctypes.byref(v)) == mhd.MHD_EINVAL
