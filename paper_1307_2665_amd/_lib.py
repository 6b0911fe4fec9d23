"""ctypes declarations of include/hps.h and the loader of libhps.so.

The library is opened on first use, so that importing the package (for
instance to run ``python -m paper_1307_2665_amd.build_lib`` on a clean tree)
does not need it.  There is no fallback: the first call into a missing
library raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HPS_LIB", os.path.join(HERE, "libhps.so"))

HPS_OK, HPS_EINVAL, HPS_ESINGULAR, HPS_ENOMEM, HPS_EDEVICE, HPS_ENOTCONV, HPS_ESURROGATE = range(7)
HPS_FP64, HPS_MIXED_SPLIT32, HPS_SURROGATE, HPS_MIXED_BF16X6 = 0, 1, 2, 3
STATUS_NAMES = {0: "HPS_OK", 1: "HPS_EINVAL", 2: "HPS_ESINGULAR", 3: "HPS_ENOMEM",
                4: "HPS_EDEVICE", 5: "HPS_ENOTCONV", 6: "HPS_ESURROGATE"}


class BuildOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("stream", C.c_void_p), ("device_ptrs", C.c_int),
                ("keep_leaf_ops", C.c_int), ("keep_factors", C.c_int),
                ("compute_root_dtn", C.c_int), ("pivot_tol", C.c_double),
                ("surrogate", C.c_void_p), ("judge_samples", C.c_int), ("judge_tol", C.c_double),
                ("keep_leaf_solution", C.c_int), ("keep_body_operator", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("device_ptrs", C.c_int), ("refine", C.c_int),
                ("refine_tol", C.c_double), ("max_iter", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("last_update_rel", C.c_double),
                ("first_update_rel", C.c_double), ("n_fallback_leaves", C.c_int)]


class OpInfo(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("p", C.c_int), ("q", C.c_int), ("N", C.c_int),
                ("n_bdry", C.c_int), ("n_boxes", C.c_int), ("n_levels", C.c_int),
                ("mode", C.c_int), ("n_fallback_leaves", C.c_int), ("box", C.c_double * 4),
                ("bytes_S", C.c_int64), ("bytes_total", C.c_int64), ("flops_build", C.c_int64),
                ("judge_worst", C.c_double), ("n_judged", C.c_int)]


class Problem(C.Structure):
    _fields_ = [("coeffs", C.c_void_p), ("box", C.c_double * 4), ("nleaf", C.c_int * 2),
                ("p", C.c_int), ("q", C.c_int)]


class HpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


P = C.c_void_p
I = C.c_int
D = C.c_double
IP = C.POINTER(C.c_int)

# name -> argtypes (restype is hps_status = int unless stated)
SIGNATURES = {
    "hps_cheb_nodes": [P, P, I, P],
    "hps_gauss_nodes_grid": [P, P, I, P, IP],
    "hps_boundary_ids": [P, I, P, IP],
    "hps_leaf_dtn": [P, I, D, D, I, I, P, P],
    "hps_build_solution_operator": [P, P, P, I, I, C.POINTER(BuildOpts), C.POINTER(P)],
    "hps_gauss_nodes": [P, P, IP],
    "hps_boundary_nodes": [P, P, IP],
    "hps_solve": [P, P, I, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo)],
    "hps_root_dtn_apply": [P, P, I, P, C.POINTER(SolveOpts)],
    "hps_postprocess": [P, P, I, P, C.POINTER(SolveOpts)],
    "hps_solve_body": [P, P, P, I, P, P, C.POINTER(SolveOpts)],
    "hps_interface_residual": [P, P, I, P, P],
    "hps_interface_residual_noalloc": [P, P, I, P, P],
    "hps_bgj_fallbacks": [C.POINTER(C.c_longlong)],
    "hps_solve_with_sources": [P, P, P, I, P, P],
    "hps_build_batch": [C.POINTER(Problem), I, C.POINTER(BuildOpts), C.POINTER(P)],
    "hps_solve_batch": [P, I, P, P, P, C.POINTER(SolveOpts)],
    "hps_op_query": [P, C.POINTER(OpInfo)],
    "hps_box": [P, I, P],
    "hps_export_S": [P, I, P, IP, IP],
    "hps_export_root_dtn": [P, P],
    "hps_export_leaf_dtn": [P, I, P],
    "hps_leaf_tables": [I, I, D, D, P, P, P, P, P, P, P, P],
    "hps_batched_solve": [P, P, I, I, I, P, P],
    "hps_batched_gemm": [P, P, P, I, I, I, I, D, I, P],
    "hps_hbs_sizes": [I, I, I, P, P],
    "hps_hbs_compress": [I, I, I, P, I, P, P, P, P],
    "hps_root_dtn_compress": [P, I, I, P, P, P, P],
    "hps_hbs_apply": [I, I, I, P, P, P, I, P],
    "hps_hbs_invert": [I, I, I, P, P, P],
    "hps_hbs_solve": [I, I, I, P, P, P, I, P],
    "hps_plan_box": [P, I, I, P, P, P, P, P, P, P, IP],
    "hps_tune_set": [C.c_char_p, I],
    "hps_autotune": [C.POINTER(Problem), I, P, C.POINTER(D)],
    "hps_level_conditions": [P, P, IP],
    "hps_tune_save": [C.c_char_p],
    "hps_tune_load": [C.c_char_p],
    "hps_tune_reset": [],
    "hps_surrogate_create": [I, I, D, D, I, I, C.c_ulonglong, P, C.POINTER(P)],
    "hps_surrogate_train": [P, P, P, I, I, I, D, C.c_ulonglong, P, C.POINTER(D), P],
    "hps_surrogate_grad": [P, P, P, I, P, C.POINTER(D), P],
    "hps_surrogate_predict": [P, P, I, P, P],
    "hps_surrogate_info": [P, P, C.POINTER(D)],
    "hps_surrogate_get_state": [P, P, C.POINTER(C.c_size_t)],
    "hps_surrogate_set_state": [P, P, C.c_size_t, P],
    "hps_surrogate_save": [P, C.c_char_p],
    "hps_surrogate_load": [C.c_char_p, P, C.POINTER(P)],
    "hps_mem_trim": [C.POINTER(C.c_size_t)],
    "hps_mem_stats": [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
    "hps_prof_enable": [C.c_uint],
    "hps_prof_reset": [],
    "hps_prof_query": [I, C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.POINTER(C.c_double),
                       C.POINTER(C.c_double)],
}
VOID_FUNCS = {"hps_destroy": [P], "hps_surrogate_destroy": [P]}
STR_FUNCS = {"hps_last_error": [], "hps_version": []}


def load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is not built; run `python -m paper_1307_2665_amd.build_lib` "
            "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name, args in VOID_FUNCS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None
    for name, args in STR_FUNCS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_char_p
    return lib


class _LazyLib:
    """Stands in for the CDLL until the first attribute access opens it."""

    def __init__(self):
        self._cdll = None

    def __getattr__(self, name):
        if self._cdll is None:
            self._cdll = load()
        return getattr(self._cdll, name)

    @property
    def loaded(self) -> bool:
        return self._cdll is not None


lib = _LazyLib()


def check(status: int) -> None:
    if status != HPS_OK:
        raise HpsError(status, lib.hps_last_error().decode())
