"""ctypes binding of the C ABI in include/shoot.h (argument marshalling only).

The shared library is built in-tree (``paper_2106_08817_amd/libshoot.so``) by
``__graft_entry__.build()``. There is no fallback: if the library is missing,
loading raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int32, c_size_t, c_uint32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libshoot.so")

SHOOT_OK = 0
SHOOT_E_ARG = -1
SHOOT_E_SHAPE = -2
SHOOT_E_WORKSPACE = -3
SHOOT_E_BUDGET = -4
SHOOT_E_HIP = -5
SHOOT_E_STATE = -6
SHOOT_E_IO = -7
STATUS_NAMES = {
    SHOOT_OK: "SHOOT_OK",
    SHOOT_E_ARG: "SHOOT_E_ARG",
    SHOOT_E_SHAPE: "SHOOT_E_SHAPE",
    SHOOT_E_WORKSPACE: "SHOOT_E_WORKSPACE",
    SHOOT_E_BUDGET: "SHOOT_E_BUDGET",
    SHOOT_E_HIP: "SHOOT_E_HIP",
    SHOOT_E_STATE: "SHOOT_E_STATE",
    SHOOT_E_IO: "SHOOT_E_IO",
}

SHOOT_FULL_STORE = 1
SHOOT_UNFUSED = 2
SHOOT_NO_GRAPH = 4
SHOOT_FORCE_GLOBAL_SCATTER = 8
SHOOT_SCHEME_EULERIAN = 16
SHOOT_SCHEME_MIXED = 32
SHOOT_CHECK_FINITE = 64
SHOOT_MAX_LANES = 8
SHOOT_LANES_MASK = 15 << 8


def SHOOT_LANES(n: int) -> int:
    """Plan flag fixing the number of concurrent lanes (1 <= n <= 8)."""
    return (int(n) & 15) << 8

SHOOT_TUNE_COUNT = 6

# Every function the header declares, with its ctypes signature.
EXPORTS = {
    "shoot_version": (c_char_p, []),
    "shoot_last_error": (c_char_p, []),
    "shoot_plan_create": (c_int32, [c_void_p, c_int32, c_int32, c_uint32, c_size_t, POINTER(c_void_p)]),
    "shoot_plan_workspace_bytes": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "shoot_plan_waves": (c_int32, [c_void_p, POINTER(c_int32)]),
    "shoot_plan_lanes": (c_int32, [c_void_p, POINTER(c_int32)]),
    "shoot_plan_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "shoot_plan_bind_scratch": (c_int32, [c_void_p, c_void_p]),
    "shoot_autotune": (c_int32, [c_void_p, c_void_p]),
    "shoot_plan_get_tuning": (c_int32, [c_void_p, POINTER(c_int32)]),
    "shoot_plan_set_tuning": (c_int32, [c_void_p, POINTER(c_int32)]),
    "shoot_plan_set_active": (c_int32, [c_void_p, POINTER(c_int32), c_void_p]),
    "shoot_plan_tune_class": (c_int32, [c_void_p, c_char_p, c_size_t]),
    "shoot_autotune_cached": (c_int32, [c_void_p, c_char_p, POINTER(c_int32), c_void_p]),
    "shoot_forward": (c_int32, [c_void_p, c_void_p]),
    "shoot_cost": (c_int32, [c_void_p, c_void_p]),
    "shoot_grad_p0": (c_int32, [c_void_p, c_void_p]),
    "shoot_descend": (c_int32, [c_void_p, c_float, c_int32, c_void_p]),
    "shoot_lbfgs_create": (c_int32, [c_void_p, c_int32, c_float, c_int32, POINTER(c_void_p)]),
    "shoot_lbfgs_workspace_bytes": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "shoot_lbfgs_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "shoot_lbfgs_step": (c_int32, [c_void_p, c_void_p]),
    "shoot_lbfgs_last_step": (c_int32, [c_void_p, POINTER(ctypes.c_double), POINTER(c_int32)]),
    "shoot_lbfgs_destroy": (c_int32, [c_void_p]),
    "shoot_plan_displacements": (c_int32, [c_void_p, POINTER(c_float), c_void_p]),
    "shoot_stream_copy": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "shoot_plan_set_profiling": (c_int32, [c_void_p, c_int32]),
    "shoot_plan_reset_stats": (c_int32, [c_void_p]),
    "shoot_plan_kernel_stats": (c_int32, [c_void_p, c_int32, POINTER(c_char_p), POINTER(ctypes.c_int64),
                                          POINTER(ctypes.c_double)]),
    "shoot_plan_destroy": (c_int32, [c_void_p]),
}


class ShootPair(ctypes.Structure):
    """Mirror of ``struct shoot_pair``."""

    _fields_ = [
        ("ndim", c_int32),
        ("shape", c_int32 * 3),
        ("rho", c_float),
        ("sigma", c_float),
        ("lambda_", c_float),
        ("image", c_void_p),
        ("target", c_void_p),
        ("p0", c_void_p),
        ("out_image", c_void_p),
        ("out_momentum", c_void_p),
        ("out_grad", c_void_p),
        ("out_cost", c_void_p),
        ("out_deformation", c_void_p),
    ]


class ShootError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_LIB = None


def load() -> ctypes.CDLL:
    """Load libshoot.so once; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(status: int, where: str) -> None:
    if status != SHOOT_OK:
        msg = load().shoot_last_error()
        raise ShootError(status, where, msg.decode() if msg else "")
