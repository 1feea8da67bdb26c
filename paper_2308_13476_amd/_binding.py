"""ctypes binding of libhelmg.so (include/helmg.h): argument marshalling only.

Every numerical step runs in the HIP library; this module passes PyTorch
device pointers and the current HIP stream. It fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libhelmg.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_E_ARG, MG_E_HIP, MG_E_DIVERGED, MG_E_WORKSPACE, MG_E_STATE = -1, -2, -3, -4, -5
MG_TRANSFER_BEZIER, MG_TRANSFER_LINEAR = 0, 1
MG_V, MG_W = 1, 2
MG_JACOBI, MG_GMRES3 = 0, 1
MG_FP64, MG_FP32_REFINED = 0, 1

EXPORTED = [
    "mg_workspace_bytes", "mg_setup", "mg_update_k2", "mg_solve", "mg_solve_multi", "mg_tune",
    "mg_fgmres_workspace_bytes", "mg_solve_fgmres", "mg_grad", "mg_destroy",
    "mg_status_string", "mg_last_error", "mg_level_info", "mg_get_stencil", "mg_apply", "mg_residual",
    "mg_residual_noalloc",
    "mg_smooth", "mg_restrict", "mg_prolong_add", "mg_coarse_solve", "mg_cycle", "mg_set_timing",
    "mg_get_timing",
]


class SetupOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_batch", ctypes.c_int), ("coarsest_n", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("tune_cache", ctypes.c_char_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("omega", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int), ("divergence", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.POINTER(ctypes.c_int)), ("relres", ctypes.POINTER(ctypes.c_double)),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("seconds", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("block_cap", ctypes.c_int), ("tail_n", ctypes.c_int), ("level1_product", ctypes.c_int),
                ("ms_per_cycle", ctypes.c_double), ("candidates", ctypes.c_int), ("tall_rows", ctypes.c_int),
                ("small_rows", ctypes.c_int), ("from_cache", ctypes.c_int)]


class MGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_13476_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    pi, pd = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "mg_workspace_bytes": (sz, [ci, ci, ci, ctypes.POINTER(SetupOpts)]),
        "mg_setup": (ci, [vp, ci, cd, cd, ci, ci, ctypes.POINTER(SetupOpts), vp, sz, vp, ctypes.POINTER(vp)]),
        "mg_update_k2": (ci, [vp, vp, vp]),
        "mg_solve": (ci, [vp, vp, vp, ci, cd, ci, ci, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]),
        "mg_solve_multi": (ci, [ctypes.POINTER(vp), ci, ctypes.POINTER(vp), ctypes.POINTER(vp), pi, cd, ci, ci,
                                ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]),
        "mg_tune": (ci, [vp, vp, ci, ci, ci, ctypes.POINTER(SolveOpts), ctypes.POINTER(TuneResult), vp]),
        "mg_fgmres_workspace_bytes": (sz, [vp, ci]),
        "mg_solve_fgmres": (ci, [vp, vp, vp, ci, cd, ci, ci, ci, ctypes.POINTER(SolveOpts), vp, sz,
                                 ctypes.POINTER(SolveStats), vp]),
        "mg_grad": (ci, [vp, vp, vp, ci, cd, ci, ci, ctypes.POINTER(SolveOpts), vp, vp,
                         ctypes.POINTER(SolveStats), vp]),
        "mg_destroy": (ci, [vp]),
        "mg_status_string": (ctypes.c_char_p, [ci]),
        "mg_last_error": (ctypes.c_char_p, [vp]),
        "mg_level_info": (ci, [vp, ci, pi, pi, pi]),
        "mg_get_stencil": (ci, [vp, ci, vp, vp]),
        "mg_apply": (ci, [vp, ci, vp, vp, ci, ci, vp]),
        "mg_residual": (ci, [vp, ci, vp, vp, vp, ci, ci, vp]),
        "mg_residual_noalloc": (ci, [vp, ci, vp, vp, vp, ci, ci, vp]),
        "mg_smooth": (ci, [vp, ci, ci, ci, cd, vp, vp, ci, ci, vp]),
        "mg_restrict": (ci, [vp, ci, vp, vp, ci, ci, vp]),
        "mg_prolong_add": (ci, [vp, ci, vp, vp, ci, ci, vp]),
        "mg_coarse_solve": (ci, [vp, vp, vp, ci, ci, vp]),
        "mg_cycle": (ci, [vp, vp, vp, ci, ci, ci, ctypes.POINTER(SolveOpts), vp]),
        "mg_set_timing": (ci, [vp, ci]),
        "mg_get_timing": (ci, [vp, pi, pd, pd]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_string(status: int) -> str:
    try:
        return lib().mg_status_string(status).decode()
    except Exception:  # pragma: no cover - only for messages
        return str(status)


def last_error(handle) -> str:
    msg = lib().mg_last_error(handle)
    return msg.decode() if msg else ""
