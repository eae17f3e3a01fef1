"""ctypes declarations of the C ABI in include/psca.h.

Loading fails loudly: there is no CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpsca.so")

PSCA_OK = 0
PSCA_EINVAL = -1
PSCA_ENOTPD = -2
PSCA_EHIP = -3
PSCA_ENOMEM = -4
PSCA_ENOTSUP = -5
PSCA_ESYNC = -6

ML_K, MAP_K, ML_UD, MAP_UR, MAP_K2 = 0, 1, 2, 3, 4
DIST_AREA, DIST_LINEAR = 0, 1   # psca_params.dist_law
MAX_L = 256

# every symbol include/psca.h declares
EXPORTED = (
    "psca_version", "psca_strerror", "psca_create", "psca_destroy", "psca_sample_cov", "psca_sample_cov_batch",
    "psca_detect", "psca_detect_y", "psca_iterate", "psca_threshold", "psca_detect_batch",
    "psca_autotune_batch", "psca_plan_create", "psca_plan_launch", "psca_plan_team_size", "psca_plan_destroy",
    "psca_net_forward", "psca_layer_backward", "psca_layer_backward_batch", "psca_detect_noalloc",
)


class PscaParams(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("rho0", ctypes.c_float),
        ("rho_decay", ctypes.c_float),
        ("rho", ctypes.c_void_p),
        ("sigma2", ctypes.c_float),
        ("M", ctypes.c_int32),
        ("g", ctypes.c_void_p),
        ("p", ctypes.c_void_p),
        ("d_lo", ctypes.c_float),
        ("d_hi", ctypes.c_float),
        ("pl_c0", ctypes.c_float),
        ("pl_beta", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("c1", ctypes.c_void_p),
        ("c2_ptr", ctypes.c_void_p),
        ("c2_col", ctypes.c_void_p),
        ("c2_val", ctypes.c_void_p),
        ("c2_nnz", ctypes.c_int32),
        ("dist_law", ctypes.c_int32),
        ("x0", ctypes.c_void_p),
    ]


class PscaProblem(ctypes.Structure):
    _fields_ = [
        ("Sigma_hat", ctypes.c_void_p),
        ("S", ctypes.c_void_p),
        ("L", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("prm", PscaParams),
        ("x_out", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("x_hist", ctypes.c_void_p),
    ]


class PscaBackProblem(ctypes.Structure):
    _fields_ = [
        ("Sigma_hat", ctypes.c_void_p),
        ("S", ctypes.c_void_p),
        ("L", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("prm", PscaParams),
        ("x_in", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("grad_x", ctypes.c_void_p),
        ("grad_rho", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


class PscaError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpsca.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2503_15259_amd.build` "
            "(this package has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
    P = ctypes.POINTER(PscaParams)
    sig = {
        "psca_version": ([], i32),
        "psca_strerror": ([i32], ctypes.c_char_p),
        "psca_create": ([ctypes.POINTER(vp), i32], i32),
        "psca_destroy": ([vp], i32),
        "psca_sample_cov": ([vp, vp, i32, i32, vp, vp], i32),
        "psca_sample_cov_batch": ([vp, i32, vp, ctypes.c_longlong, i32, i32, vp, ctypes.c_longlong, vp], i32),
        "psca_detect": ([vp, vp, vp, i32, i32, P, vp, vp, vp], i32),
        "psca_detect_y": ([vp, vp, vp, i32, i32, P, vp, vp, vp], i32),
        "psca_detect_noalloc": ([vp, vp, vp, i32, i32, P, vp, vp, vp], i32),
        "psca_iterate": ([vp, vp, vp, i32, i32, P, f32, vp, vp, vp, vp, vp, vp, vp], i32),
        "psca_threshold": ([vp, i32, f32, vp, vp], i32),
        "psca_detect_batch": ([vp, i32, ctypes.POINTER(PscaProblem), vp], i32),
        "psca_autotune_batch": ([vp, i32, ctypes.POINTER(PscaProblem), i32, ctypes.POINTER(i32), vp], i32),
        "psca_plan_create": ([vp, i32, ctypes.POINTER(PscaProblem), i32, ctypes.POINTER(vp)], i32),
        "psca_plan_launch": ([vp, vp], i32),
        "psca_plan_team_size": ([vp], i32),
        "psca_plan_destroy": ([vp], i32),
        "psca_net_forward": ([vp, vp, vp, i32, i32, P, vp, vp, vp], i32),
        "psca_layer_backward": ([vp, vp, vp, i32, i32, P, f32, vp, vp, vp, vp, vp, vp], i32),
        "psca_layer_backward_batch": ([vp, i32, ctypes.POINTER(PscaBackProblem), f32, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().psca_strerror(code).decode()


def check(code: int, what: str) -> None:
    if code != PSCA_OK:
        raise PscaError(code, what)
