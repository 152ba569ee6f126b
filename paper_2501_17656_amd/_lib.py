"""ctypes declarations of the C ABI in include/h2mg.h.

Loading fails loudly when libh2mg.so has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libh2mg.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P_double = ctypes.POINTER(c_double)
P_int64 = ctypes.POINTER(c_int64)
P_int32 = ctypes.POINTER(c_int32)


class Kernel(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("length_scale", c_double), ("shift", c_double),
                ("derivative", c_int32)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_size", c_int32), ("eta", c_double), ("cheb_m", c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("n_fine", c_int32), ("n_coarse", c_int32), ("rtol", c_double),
                ("max_cycles", c_int32), ("precision", c_int32), ("use_x0", c_int32),
                ("smoother", c_int32), ("method", c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", c_int32), ("converged", c_int32), ("rel_residual", c_double),
                ("solve_seconds", c_double), ("history_len", c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("dim", c_int32), ("depth", c_int32), ("d_top", c_int32),
                ("rank", c_int32), ("leaf_min", c_int32), ("leaf_max", c_int32)]


STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "HIP", 4: "NOT_SPD",
          5: "NOT_CONVERGED", 6: "NUMERIC", 7: "STATE"}

# name -> (restype, argtypes)
SIGNATURES = {
    "h2mg_plan_create": (c_int32, [c_void_p, c_int64, c_int32, ctypes.POINTER(BuildOpts), ctypes.POINTER(c_void_p)]),
    "h2mg_plan_query": (c_int32, [c_void_p, ctypes.POINTER(PlanInfo)]),
    "h2mg_plan_perm": (c_int32, [c_void_p, c_void_p]),
    "h2mg_plan_offsets": (c_int32, [c_void_p, c_int32, c_void_p]),
    "h2mg_plan_pair_count": (c_int32, [c_void_p, c_int32, c_int32, P_int64]),
    "h2mg_plan_pairs": (c_int32, [c_void_p, c_int32, c_int32, c_void_p]),
    "h2mg_plan_destroy": (None, [c_void_p]),
    "h2mg_build": (c_int32, [c_void_p, c_int64, c_int32, ctypes.POINTER(Kernel), ctypes.POINTER(BuildOpts),
                             c_void_p, ctypes.POINTER(c_void_p)]),
    "h2mg_matvec": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "h2mg_setup_mg": (c_int32, [c_void_p, c_int32, c_void_p]),
    "h2mg_level_count": (c_int32, [c_void_p, P_int32]),
    "h2mg_level_size": (c_int32, [c_void_p, c_int32, P_int64]),
    "h2mg_level_apply": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "h2mg_level_apply_precision": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "h2mg_restrict": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "h2mg_prolong": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "h2mg_vcycle": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts), c_void_p]),
    "h2mg_solve": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts),
                             ctypes.POINTER(SolveInfo), c_void_p]),
    "h2mg_solve_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(SolveInfo), c_void_p]),
    "h2mg_solve_history": (c_int32, [c_void_p, P_double, c_int32]),
    "h2mg_memory_bytes": (c_int32, [c_void_p, P_int64]),
    "h2mg_gemv_launch_info": (c_int32, [c_void_p, c_int32, P_int64, P_int64]),
    "h2mg_set_timing": (c_int32, [c_void_p, c_int32]),
    "h2mg_store_near": (c_int32, [c_void_p, c_int32, c_void_p]),
    "h2mg_set_graphs": (c_int32, [c_void_p, c_int32]),
    "h2mg_set_autotune": (c_int32, [c_void_p, c_int32]),
    "h2mg_block_tuning": (c_int32, [c_void_p, c_int32, P_int32, P_double, P_int64]),
    "h2mg_matvec_multi": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_int32, c_void_p]),
    "h2mg_solve_multi": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_int32,
                                   ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), P_double, c_void_p]),
    "h2mg_solve_batch": (c_int32, [c_int32, ctypes.POINTER(c_void_p), P_int32, ctypes.POINTER(c_void_p), P_int32,
                                   ctypes.POINTER(c_void_p), P_int32, ctypes.POINTER(SolveOpts),
                                   ctypes.POINTER(SolveInfo), P_int32, c_int32, c_void_p]),
    "h2mg_solve_group": (c_int32, [c_int32, ctypes.POINTER(c_void_p), P_int32, ctypes.POINTER(c_void_p), P_int32,
                                   ctypes.POINTER(c_void_p), P_int32, ctypes.POINTER(SolveOpts),
                                   ctypes.POINTER(SolveInfo), P_int32, c_void_p]),
    "h2mg_build_scaled": (c_int32, [c_void_p, c_int64, c_int32, ctypes.POINTER(Kernel), ctypes.POINTER(BuildOpts),
                                    c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "h2mg_bem_panels": (c_int32, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "h2mg_bem_point_source_rhs": (c_int32, [c_void_p, c_void_p, c_int64, P_double, c_void_p, c_void_p]),
    "h2mg_bem_quadrature7": (c_int32, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "h2mg_set_near_quadrature": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "h2mg_bem_density": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "h2mg_bem_harmonic_rhs": (c_int32, [c_void_p, c_void_p, c_int64, P_double, c_void_p, c_void_p]),
    "h2mg_smooth": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p]),
    "h2mg_build_derivative": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(c_void_p)]),
    "h2mg_quadratic_gradient": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                          P_double, P_double, P_double, c_void_p, c_void_p, c_void_p]),
    "h2mg_kernel_stats": (c_int32, [c_void_p, c_int32, P_int64, P_double, P_double]),
    "h2mg_destroy": (c_int32, [c_void_p]),
    "h2mg_last_error": (ctypes.c_char_p, []),
}


class H2MGError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


_lib = None


def lib():
    """The loaded library (raises if libh2mg.so is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2501_17656_amd.build` (no fallback exists)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def last_error() -> str:
    msg = lib().h2mg_last_error()
    return msg.decode() if msg else ""


def check(status: int, message: str = None) -> None:
    """Raise H2MGError for a failed call (message: the error text read right
    after that call, when other calls have been made since)."""
    if status != 0:
        raise H2MGError(status, last_error() if message is None else message)
