"""ctypes loader of libccmf.so: argument marshalling only, no arithmetic."""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libccmf.so")

# return codes of include/ccmf.h
CCMF_OK = 0
CCMF_NOT_CONVERGED = 1
CCMF_EINVAL = -1
CCMF_ENOMEM = -2
CCMF_EDEVICE = -3
CCMF_ESTATE = -4
CCMF_F64 = 0
CCMF_F32 = 1
RULES = {"bb": 0, "const": 1, "ltd": 2}

EXPORTS = ("ccmf_setup", "ccmf_solve", "ccmf_grad_kappa", "ccmf_certificate", "ccmf_mean_flux", "ccmf_get_state",
           "ccmf_set_state", "ccmf_history", "ccmf_kernel_times", "ccmf_laplace_pinv", "ccmf_hartley_axis", "ccmf_stream_copy",
           "ccmf_destroy", "ccmf_last_error")


class Options(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("rho0", ctypes.c_double), ("rule", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32), ("bb_min_corr", ctypes.c_double),
                ("eta0", ctypes.c_double), ("k0", ctypes.c_double), ("eager", ctypes.c_int32),
                ("no_autotune", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("record_history", ctypes.c_int32)]


class CcmfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ccmf error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it first (python -m paper_2103_05968_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    pd, pi32, pi64 = ctypes.POINTER(dbl), ctypes.POINTER(i32), ctypes.POINTER(i64)
    lib.ccmf_setup.argtypes = [ctypes.POINTER(vp), pi64, i64, i32, vp, vp]
    lib.ccmf_solve.argtypes = [vp, pd, i64, dbl, ctypes.POINTER(Options), pd, pi32, pd, pd, vp, vp]
    lib.ccmf_grad_kappa.argtypes = [vp, pd, vp]
    lib.ccmf_kernel_times.argtypes = [vp, pd, pi64, pd]
    lib.ccmf_certificate.argtypes = [vp, pd, pd]
    lib.ccmf_mean_flux.argtypes = [vp, pd]
    lib.ccmf_get_state.argtypes = [vp, vp, vp, pd, pi32]
    lib.ccmf_set_state.argtypes = [vp, i64, vp, vp, pd, pi32]
    lib.ccmf_history.argtypes = [vp, i32, pd]
    lib.ccmf_laplace_pinv.argtypes = [vp, vp, vp, i64]
    lib.ccmf_hartley_axis.argtypes = [vp, vp, i64, i32]
    lib.ccmf_stream_copy.argtypes = [vp, vp, i64, vp]
    lib.ccmf_destroy.argtypes = [vp]
    lib.ccmf_destroy.restype = None
    lib.ccmf_last_error.restype = ctypes.c_char_p
    for name in ("ccmf_setup", "ccmf_solve", "ccmf_grad_kappa", "ccmf_certificate", "ccmf_mean_flux",
                 "ccmf_get_state", "ccmf_set_state", "ccmf_history", "ccmf_kernel_times", "ccmf_laplace_pinv",
                 "ccmf_hartley_axis", "ccmf_stream_copy"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def check(code, allow_not_converged=False):
    if code == CCMF_OK or (allow_not_converged and code == CCMF_NOT_CONVERGED):
        return code
    msg = load().ccmf_last_error().decode(errors="replace")
    raise CcmfError(code, msg)
