"""ctypes view of libfcgle.so (the C ABI of include/fcgle.h).

torch is imported first so that the library binds to the same HIP runtime as
torch's streams and allocator.  There is no fallback: if the library is missing
this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library must share)

HERE = os.path.dirname(os.path.abspath(__file__))
# FCGLE_LIB selects another build of the same library (the host-sanitizer build of build.py)
LIB_PATH = os.environ.get("FCGLE_LIB") or os.path.join(HERE, "libfcgle.so")

c_int = ctypes.c_int
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
P_i64 = ctypes.POINTER(ctypes.c_int64)
P_dbl = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [("nu", c_dbl), ("eta", c_dbl), ("gamma", c_dbl), ("kappa", c_dbl), ("zeta", c_dbl)]


# status codes
OK, ERR_ARG, ERR_UNSUPPORTED, ERR_NOMEM, ERR_HIP, ERR_NONFINITE, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
KINDS = {"inv": 0, "exp": 1, "phi1": 2, "phi2": 3, "phi3": 4}
SCHEMES = {"exp_euler": 0, "lawson": 1, "lie": 2, "lbdf2": 3, "strang": 4, "krogstad": 5}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}

# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("fcgle_setup", c_int, [c_int, P_i64, P_dbl, P_dbl, ctypes.POINTER(Params), c_int, c_int, c_dbl,
                            ctypes.POINTER(c_vp)]),
    ("fcgle_destroy", None, [c_vp]),
    ("fcgle_last_error", ctypes.c_char_p, []),
    ("fcgle_get_eig", c_int, [c_vp, c_int, P_dbl, P_dbl]),
    ("fcgle_set_source", c_int, [c_vp, c_int, P_dbl, P_dbl, ctypes.POINTER(c_vp)]),
    ("fcgle_apply_f", c_int, [c_vp, c_int, c_dbl, c_vp, c_vp, c_vp]),
    ("fcgle_apply_f_noalloc", c_int, [c_vp, c_int, c_dbl, c_vp, c_vp, c_vp]),
    ("fcgle_apply_inv_refined", c_int, [c_vp, c_dbl, c_vp, c_vp, c_int, P_dbl, c_vp]),
    ("fcgle_set_state", c_int, [c_vp, c_vp, c_vp, c_vp]),
    ("fcgle_step", c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_vp]),
    ("fcgle_run", c_int, [c_vp, c_int, c_vp, c_dbl, c_dbl, c_i64, c_vp]),
    ("fcgle_vjp", c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_dbl, c_dbl, c_vp]),
    ("fcgle_vjp_run", c_int, [c_vp, c_int, c_vp, c_i64, c_vp, c_vp, c_dbl, c_dbl, c_vp]),
    ("fcgle_check_finite", c_int, [c_vp, c_vp, c_vp]),
    ("fcgle_plan_shape", c_int, [c_vp, P_i64, ctypes.POINTER(c_int)]),
    ("fcgle_autotune", c_int, [c_vp, c_int, c_vp]),
    ("fcgle_set_tiles", c_int, [c_vp, c_int, c_int, c_int]),
    ("fcgle_set_fusion", c_int, [c_vp, c_int]),
    ("fcgle_set_structure", c_int, [c_vp, c_int]),
    ("fcgle_set_wide_loads", c_int, [c_vp, c_int]),
    ("fcgle_describe", c_int, [c_vp, ctypes.c_char_p, ctypes.c_size_t]),
    ("fcgle_timing_enable", c_int, [c_vp, c_int]),
    ("fcgle_timing_read", c_int, [c_vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                  ctypes.POINTER(c_int), P_dbl, P_i64]),
    ("fcgle_batch_setup", c_int, [c_int, P_i64, P_dbl, P_dbl, ctypes.POINTER(Params), c_int, c_dbl,
                                  ctypes.POINTER(c_vp)]),
    ("fcgle_batch_run", c_int, [c_vp, c_int, ctypes.POINTER(c_vp), c_dbl, c_dbl, c_i64, c_vp]),
    ("fcgle_batch_set_persistent", c_int, [c_vp, c_int, c_i64]),
    ("fcgle_host_fd_weights", c_int, [c_dbl, c_i64, c_int, P_dbl]),
    ("fcgle_host_eig", c_int, [c_i64, c_dbl, c_dbl, c_int, P_dbl, P_dbl]),
    ("fcgle_host_fz", c_int, [c_int, c_i64, P_dbl, P_dbl]),
]


class FcgleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fcgle error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the shared library (once) and declare its prototypes."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_21394_amd.build` "
                              "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int) -> int:
    if code != OK:
        msg = lib().fcgle_last_error()
        raise FcgleError(code, msg.decode() if msg else "")
    return code
