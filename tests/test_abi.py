"""The C-ABI library loads and exports every entry point include/ccmf.h declares
(no compute call: runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccmf.h")
LIB = os.path.join(ROOT, "paper_2103_05968_amd", "libccmf.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ccmf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for want in ("ccmf_setup", "ccmf_solve", "ccmf_grad_kappa", "ccmf_destroy", "ccmf_last_error"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    from paper_2103_05968_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_paths_without_device():
    """Argument validation happens before any device call."""
    from paper_2103_05968_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 3)(4, 0, 4)
    assert lib.ccmf_setup(ctypes.byref(h), dims, 1, 0, ctypes.c_void_p(1), None) == _lib.CCMF_EINVAL
    assert b"dims[1]" in lib.ccmf_last_error()
    dims = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.ccmf_setup(ctypes.byref(h), dims, 1, 7, ctypes.c_void_p(1), None) == _lib.CCMF_EINVAL
    assert lib.ccmf_solve(None, None, 1, 1e-4, None, None, None, None, None, None, None) == _lib.CCMF_EINVAL
    assert lib.ccmf_stream_copy(ctypes.c_void_p(1), ctypes.c_void_p(1), 15, None) == _lib.CCMF_EINVAL
    # entry points that take a plan reject a null plan before touching the device
    d = ctypes.c_double()
    assert lib.ccmf_grad_kappa(None, ctypes.byref(d), ctypes.c_void_p(1)) == _lib.CCMF_EINVAL
    assert lib.ccmf_certificate(None, ctypes.byref(d), None) == _lib.CCMF_EINVAL
    assert lib.ccmf_mean_flux(None, ctypes.byref(d)) == _lib.CCMF_EINVAL
    assert lib.ccmf_get_state(None, None, None, None, None) == _lib.CCMF_EINVAL
    k = ctypes.c_int32()
    assert lib.ccmf_set_state(None, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.byref(d),
                              ctypes.byref(k)) == _lib.CCMF_EINVAL
    assert lib.ccmf_laplace_pinv(None, ctypes.c_void_p(1), ctypes.c_void_p(1), 1) == _lib.CCMF_EINVAL
    assert lib.ccmf_kernel_times(None, None, None, None) == _lib.CCMF_EINVAL
    assert lib.ccmf_history(None, 1, ctypes.byref(d)) == _lib.CCMF_EINVAL
