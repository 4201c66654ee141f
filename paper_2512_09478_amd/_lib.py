"""ctypes binding of libkifmm.so (argument marshalling only).

The shared object is built in-tree by ``paper_2512_09478_amd.build``; there is
no fallback: if it is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkifmm.so")

KIFMM_LAPLACE, KIFMM_GRAVITY = 0, 1
KIFMM_FP32, KIFMM_SPLIT_BF16 = 0, 1
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_INPUT", -3: "ERR_OOM", -4: "ERR_HIP", -5: "ERR_STATE"}


class KifmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("adaptive", ctypes.c_int), ("max_depth", ctypes.c_int), ("precision", ctypes.c_int),
                ("pinv_rtol", ctypes.c_double), ("explicit_root", ctypes.c_int),
                ("root_lo", ctypes.c_double * 3), ("root_side", ctypes.c_double), ("profile", ctypes.c_int),
                ("periodic", ctypes.c_int), ("m2l_rtol", ctypes.c_double)]


_lock = threading.Lock()
_lib = None

EXPORTS = ["kifmm_default_options", "kifmm_setup", "kifmm_setup_ex", "kifmm_rebuild", "kifmm_set_precision",
           "kifmm_evaluate", "kifmm_evaluate_dipoles", "kifmm_evaluate_gradient", "kifmm_evaluate_stokes",
           "kifmm_evaluate_stokes_ex", "kifmm_backward",
           "kifmm_clump_reduce", "kifmm_clump_reduce_noalloc", "kifmm_clump_backward", "kifmm_set_clumps", "kifmm_clump_forces",
           "kifmm_clump_forces_backward", "kifmm_synchronize", "kifmm_get_counts", "kifmm_get_m2l_rank",
           "kifmm_get_build_stats", "kifmm_get_operator", "kifmm_copy_tree", "kifmm_copy_list", "kifmm_get_phase_times",
           "kifmm_get_phase_times_at", "kifmm_destroy", "kifmm_status_string"]


def lib():
    """Load libkifmm.so once; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_2512_09478_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
            H = ctypes.c_void_p
            L.kifmm_default_options.argtypes = [ctypes.POINTER(Options)]
            L.kifmm_default_options.restype = None
            L.kifmm_setup.argtypes = [P, I64, I, I, I, ctypes.POINTER(H)]
            L.kifmm_setup_ex.argtypes = [P, I64, I, I, I, ctypes.POINTER(Options), P, ctypes.POINTER(H)]
            L.kifmm_rebuild.argtypes = [H, P, P]
            L.kifmm_set_precision.argtypes = [H, I]
            L.kifmm_evaluate.argtypes = [H, P, P, P, P]
            L.kifmm_evaluate_dipoles.argtypes = [H, P, P, P, P, P]
            L.kifmm_evaluate_gradient.argtypes = [H, P, P, P, P, P, P]
            L.kifmm_evaluate_stokes.argtypes = [H, P, D, P, P]
            L.kifmm_evaluate_stokes_ex.argtypes = [H, P, D, P, P, P]
            L.kifmm_backward.argtypes = [H, P, P, P, P, P, P]
            L.kifmm_clump_reduce.argtypes = [H, P, P, P, I64, P, P, P, P]
            L.kifmm_clump_reduce_noalloc.argtypes = [H, P, P, P, I64, P, P, P, P]
            L.kifmm_clump_backward.argtypes = [H, P, P, P, I64, P, P, P, P, P, P, P, P]
            L.kifmm_set_clumps.argtypes = [H, P, I64, P]
            L.kifmm_clump_forces.argtypes = [H, P, P, P, P, P, P]
            L.kifmm_clump_forces_backward.argtypes = [H, P, P, P, P, P, P, P, P]
            L.kifmm_synchronize.argtypes = [H, P]
            L.kifmm_get_counts.argtypes = [H, ctypes.POINTER(I64)]
            L.kifmm_get_m2l_rank.argtypes = [H, ctypes.POINTER(I64)]
            L.kifmm_get_operator.argtypes = [H, I, P, I64, ctypes.POINTER(I64)]
            L.kifmm_get_build_stats.argtypes = [H, ctypes.POINTER(I64)]
            L.kifmm_copy_tree.argtypes = [H, P, P, P, P, P, P, P, P, P]
            L.kifmm_copy_list.argtypes = [H, ctypes.c_char, P, P]
            L.kifmm_get_phase_times.argtypes = [H, ctypes.POINTER(ctypes.c_float), I]
            L.kifmm_get_phase_times_at.argtypes = [H, I, ctypes.POINTER(ctypes.c_float), I]
            L.kifmm_destroy.argtypes = [H]
            L.kifmm_destroy.restype = None
            L.kifmm_status_string.argtypes = [I]
            L.kifmm_status_string.restype = ctypes.c_char_p
            for name in ("kifmm_setup", "kifmm_setup_ex", "kifmm_rebuild", "kifmm_set_precision",
                         "kifmm_evaluate", "kifmm_evaluate_dipoles", "kifmm_evaluate_gradient",
                         "kifmm_evaluate_stokes", "kifmm_evaluate_stokes_ex", "kifmm_backward",
                         "kifmm_clump_reduce", "kifmm_clump_reduce_noalloc", "kifmm_clump_backward", "kifmm_set_clumps", "kifmm_clump_forces",
                         "kifmm_clump_forces_backward", "kifmm_synchronize",
                         "kifmm_get_counts", "kifmm_get_m2l_rank", "kifmm_get_operator", "kifmm_get_build_stats",
                         "kifmm_copy_tree", "kifmm_copy_list", "kifmm_get_phase_times",
                         "kifmm_get_phase_times_at"):
                getattr(L, name).restype = I
            _lib = L
    return _lib


def check(code: int) -> int:
    if code < 0:
        raise KifmmError(code, lib().kifmm_status_string(code).decode())
    return code
