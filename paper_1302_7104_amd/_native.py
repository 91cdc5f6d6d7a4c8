"""ctypes binding of libpclb.so (the C ABI declared in include/pclb.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  There is no fallback: if the library is missing or fails to load,
``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpclb.so")

PCLB_OK = 0
ERRORS = {
    -1: "PCLB_EINVAL", -2: "PCLB_ECFL", -3: "PCLB_EDEVICE", -4: "PCLB_ENOMEM",
    -5: "PCLB_ESTATE", -6: "PCLB_ENONFINITE",
}
WALL, INFLOW, EXTRAPOLATE = 0, 1, 2
KERNEL_AUTO, KERNEL_NODE, KERNEL_STRIP = 0, 1, 2
ORDER_DEFAULT, ORDER_XCD, ORDER_PLAIN = 0, 1, 2
NONEQ_M, NONEQ_MSTAR, NONEQ_DELTA, NONEQ_DSTAR, NONEQ_ALL = 1, 2, 4, 8, 15
SCHEME_MWB, SCHEME_WB, SCHEME_LW, SCHEME_UPWIND2 = 0, 1, 2, 3
RELAX_ANALYTIC, RELAX_EULER = 0, 1

#: every symbol include/pclb.h declares
SYMBOLS = (
    "pclb_cfl_dt", "pclb_create", "pclb_destroy", "pclb_last_error", "pclb_bind",
    "pclb_set_bc", "pclb_init_state", "pclb_step", "pclb_step_into", "pclb_current",
    "pclb_step_count", "pclb_moments", "pclb_moments_of", "pclb_moments_host",
    "pclb_adjoint_step", "pclb_adjoint_init", "pclb_step_static", "pclb_noneq",
    "pclb_step_graph",
)


class PclbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32),
                ("r1", ctypes.c_double), ("r2", ctypes.c_double),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("n_i", ctypes.c_int32), ("n_f", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("fp64_collision", ctypes.c_int32),
                ("kernel", ctypes.c_int32),
                ("strip_chunk", ctypes.c_int32), ("strip_order", ctypes.c_int32),
                ("adjoint_tie", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("relaxation", ctypes.c_int32)]


_lib = None
_V = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libpclb.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libpclb.so not found at {LIB_PATH}: build it first (python -m "
            "paper_1302_7104_amd.build or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    C = ctypes.POINTER(Config)
    P = ctypes.c_void_p   # opaque pclb_ctx*
    L.pclb_cfl_dt.argtypes = [C, ctypes.c_double]
    L.pclb_cfl_dt.restype = ctypes.c_double
    L.pclb_create.argtypes = [C, ctypes.POINTER(ctypes.c_void_p)]
    L.pclb_destroy.argtypes = [P]
    L.pclb_destroy.restype = None
    L.pclb_last_error.argtypes = [P]
    L.pclb_last_error.restype = ctypes.c_char_p
    L.pclb_bind.argtypes = [P, _V, _V, _V]
    L.pclb_set_bc.argtypes = [P, ctypes.c_int32, ctypes.c_int32, _D]
    L.pclb_init_state.argtypes = [P, _V, _V, _V, _V]
    L.pclb_step.argtypes = [P, ctypes.c_int64]
    L.pclb_step_static.argtypes = [P, ctypes.c_int64]
    L.pclb_step_graph.argtypes = [P, ctypes.c_int64]
    L.pclb_step_into.argtypes = [P, _V, _V]
    L.pclb_current.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    L.pclb_step_count.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    L.pclb_moments.argtypes = [P, _V, _V, _V, _V, _V]
    L.pclb_moments_of.argtypes = [P, _V, _V, _V, _V, _V, _V]
    L.pclb_moments_host.argtypes = [P, _D]
    L.pclb_adjoint_step.argtypes = [P, _V, _V, _V]
    L.pclb_noneq.argtypes = [P, _V, ctypes.c_int32, _V]
    L.pclb_adjoint_init.argtypes = [P, _V, _V, _V, _V, _V, _V, _V, _V, _V]
    for name in SYMBOLS:
        if name not in ("pclb_cfl_dt", "pclb_destroy", "pclb_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int, ctx=None) -> None:
    if rc != PCLB_OK:
        msg = lib().pclb_last_error(ctx)
        raise PclbError(rc, msg.decode() if msg else "")
