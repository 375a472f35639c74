"""ctypes binding of the C ABI in include/hh.h (argument marshalling only).

The shared library ``libhh.so`` is built in place by
``paper_2308_06085_amd.build``.  Loading fails loudly when it is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhh.so")

HH_OK = 0
STATUS_NAMES = {
    0: "HH_OK",
    1: "HH_ERR_ARG",
    2: "HH_ERR_HIP",
    3: "HH_ERR_OOM",
    4: "HH_ERR_NUMERIC",
    5: "HH_ERR_BREAKDOWN",
    6: "HH_ERR_NOT_CONVERGED",
    7: "HH_ERR_STATE",
}
BC = {"dirichlet": 0, "sommerfeld": 1}
PREC = {"fp64": 0, "mixed": 1}

# every symbol include/hh.h declares
EXPORTS = [
    "hh_default_config", "hh_create", "hh_destroy", "hh_last_error", "hh_level_shape",
    "hh_set_model", "hh_set_model_slowness2", "hh_set_sources", "hh_set_point_sources", "hh_solve",
    "hh_apply_operator", "hh_apply_operator_noalloc", "hh_apply_shifted", "hh_apply_vcycle", "hh_adjoint_rhs",
    "hh_grad_slowness2", "hh_set_shadow", "hh_set_option", "hh_get_option", "hh_time_kernel", "hh_kernel_times",
    "hh_autotune",
]


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("h", C.c_double),
        ("bc", C.c_int),
        ("beta1", C.c_double), ("beta2", C.c_double),
        ("omega", C.c_double),
        ("nu_pre", C.c_int), ("nu_post", C.c_int),
        ("n_levels", C.c_int),
        ("prec", C.c_int),
        ("nrhs_max", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_double),
        ("matvecs", C.c_int),
        ("relres", C.c_double),
        ("relres_true", C.c_double),
        ("status", C.c_int),
        ("restarts", C.c_int),
        ("ms", C.c_double),
    ]


class HHError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libhh.so once and declare the signatures of every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2308_06085_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.c_double
    sig = {
        "hh_default_config": (None, [C.POINTER(Config), ip, ip, ip, dp]),
        "hh_create": (ip, [C.POINTER(Config), vp, C.POINTER(vp)]),
        "hh_destroy": (ip, [vp]),
        "hh_last_error": (C.c_char_p, [vp]),
        "hh_level_shape": (ip, [vp, ip, C.POINTER(ip), C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)]),
        "hh_set_model": (ip, [vp, vp]),
        "hh_set_model_slowness2": (ip, [vp, vp, dp]),
        "hh_set_sources": (ip, [vp, vp, ip]),
        "hh_set_point_sources": (ip, [vp, C.POINTER(ip), ip]),
        "hh_solve": (ip, [vp, vp, dp, ip, ip, C.POINTER(Stats)]),
        "hh_apply_operator": (ip, [vp, vp, vp, ip]),
        "hh_apply_operator_noalloc": (ip, [C.POINTER(Config), vp, vp, vp, ip, vp]),
        "hh_apply_shifted": (ip, [vp, vp, vp, ip]),
        "hh_apply_vcycle": (ip, [vp, vp, vp, ip]),
        "hh_adjoint_rhs": (ip, [vp, vp, vp, ip]),
        "hh_grad_slowness2": (ip, [vp, vp, vp, vp, dp, vp, ip]),
        "hh_set_shadow": (ip, [vp, vp, ip]),
        "hh_set_option": (ip, [vp, C.c_char_p, C.c_longlong]),
        "hh_get_option": (ip, [vp, C.c_char_p, C.POINTER(C.c_longlong)]),
        "hh_time_kernel": (ip, [vp, ip, ip, ip, C.POINTER(C.c_float)]),
        "hh_kernel_times": (ip, [vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
        "hh_autotune": (ip, [vp, C.c_char_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, ctx=None, allow=()):
    """Raise HHError unless status is HH_OK or in ``allow``."""
    if status == HH_OK or status in allow:
        return status
    lib = load()
    msg = lib.hh_last_error(ctx)
    raise HHError(status, msg.decode() if msg else "")
