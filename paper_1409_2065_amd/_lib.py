"""ctypes declarations for libccmi.so (the C ABI in include/ccmi.h).

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccmi.so")

CC_OK, CC_ERR_INVALID_ARG, CC_ERR_OUT_OF_MEMORY, CC_ERR_HIP, CC_ERR_NUMERIC, CC_ERR_STATE = range(6)
CC_DTYPE_F32, CC_DTYPE_F64 = 0, 1
CC_PREC_F32, CC_PREC_MIXED, CC_PREC_F64 = 0, 1, 2

i32, i64, f64, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
P_i32, P_i64, P_f64, P_u8 = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_uint8)


class SolveOpts(C.Structure):
    _fields_ = [
        ("struct_size", i32),
        ("eta", f64),
        ("rho", f64),
        ("eps", f64),
        ("tol", f64),
        ("max_iter", i32),
        ("check_every", i32),
        ("warm_start", i32),
        ("record_objective", i32),
        ("test_every", i32),
        ("proj_sweeps", i32),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", i32),
        ("converged", i32),
        ("n_clusters", i32),
        ("status", i32),
        ("gamma", f64),
        ("objective", f64),
        ("d", f64),
        ("rel_change", f64),
        ("rho", f64),
        ("eps", f64),
        ("seconds", f64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/ccmi.h
SIGNATURES = {
    "cc_status_string": (C.c_char_p, [i32]),
    "cc_last_error_message": (C.c_char_p, []),
    "cc_default_opts": (None, [C.POINTER(SolveOpts)]),
    "cc_version": (i32, []),
    "cc_problem_create": (i32, [i64, i64, i32, vp, i64, vp, i64, i64, vp, vp, vp, i32, vp, C.POINTER(vp)]),
    "cc_problem_destroy": (i32, [vp]),
    "cc_problem_dims": (i32, [vp, P_i64, P_i64, P_i64, P_i32]),
    "cc_solve": (i32, [vp, f64, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "cc_solve_path": (i32, [vp, i32, P_f64, C.POINTER(SolveOpts), vp, vp, C.POINTER(SolveInfo)]),
    "cc_get_U": (i32, [vp, i32, vp, i64]),
    "cc_get_labels": (i32, [vp, vp, P_i32]),
    "cc_get_fused_edges": (i32, [vp, vp]),
    "cc_get_trace": (i32, [vp, P_f64, i64, P_i64]),
    "cc_profile": (i32, [vp, i32]),
    "cc_kernel_stats": (i32, [vp, P_f64, P_i64]),
    "cc_state_size": (i32, [vp, C.POINTER(C.c_size_t)]),
    "cc_export_state": (i32, [vp, vp, C.c_size_t]),
    "cc_import_state": (i32, [vp, vp, C.c_size_t]),
    "cc_reset_state": (i32, [vp]),
    "cc_set_state": (i32, [vp, vp, vp, i64, vp]),
    "cc_get_state": (i32, [vp, vp, vp, i64, vp]),
    "cc_build_knn_weights": (i32, [i64, i64, i32, vp, i64, vp, i64, i32, f64, i32, vp, vp, vp, i64, P_i64, P_f64, vp]),
    "cc_standardize_columns": (i32, [i64, i64, i32, vp, i64, vp, i64, vp]),
    "cc_standardize_columns_noalloc": (i32, [i64, i64, i32, vp, i64, vp, i64, vp]),
    "cc_components": (i32, [i64, i64, vp, vp, vp, vp, P_i32, vp]),
    "cc_pca": (i32, [i64, i64, i32, vp, i64, vp, i64, i32, i32, vp, P_f64, vp, vp]),
    "cc_solve_path_pc": (i32, [vp, i32, P_f64, C.POINTER(SolveOpts), vp, i32, vp, vp, vp,
                               C.POINTER(SolveInfo)]),
    "cc_min_connected_k": (i32, [i64, i64, i32, vp, i64, vp, i64, i32, P_i32, P_i32, vp]),
    "cc_composite_weights": (i32, [i64, i64, vp, vp, i64, i32, vp, i64, vp, i64, i32, vp, i64, P_f64, i32,
                                   f64, f64, f64, i32, vp, P_f64, vp]),
    "cc_batch_create": (i32, [i32, C.POINTER(vp), P_i32, P_f64, C.POINTER(SolveOpts), i32, C.POINTER(vp)]),
    "cc_batch_run": (i32, [vp, vp, C.POINTER(SolveInfo), P_f64]),
    "cc_batch_config": (i32, [vp, P_i32, P_i32, P_i32, P_f64]),
    "cc_batch_tuning": (i32, [vp, i32, P_i32, P_i32, P_f64, P_i32]),
    "cc_batch_destroy": (i32, [vp]),
    "cc_server_create": (i32, [i32, C.POINTER(SolveOpts), i64, i32, i32, vp, C.POINTER(vp)]),
    "cc_server_submit": (i32, [vp, i64, i64, vp, vp, i32, f64, i32, P_f64, P_i64]),
    "cc_server_step": (i32, [vp, P_i32, P_i32, P_i32]),
    "cc_server_status": (i32, [vp, i64, P_i32, P_f64, P_f64, P_f64]),
    "cc_server_result": (i32, [vp, i64, vp, C.POINTER(SolveInfo), vp]),
    "cc_server_release": (i32, [vp, i64]),
    "cc_server_memory": (i32, [vp, P_i64, P_i64]),
    "cc_server_destroy": (i32, [vp]),
}

CC_REQ_WAITING, CC_REQ_ACTIVE, CC_REQ_DONE, CC_REQ_FAILED = range(4)

_lib = None


class CCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def load() -> C.CDLL:
    """Load libccmi.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libccmi.so not found at {LIB_PATH}; build it with "
            "`python -m paper_1409_2065_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_name(s: int) -> str:
    names = {0: "CC_OK", 1: "CC_ERR_INVALID_ARG", 2: "CC_ERR_OUT_OF_MEMORY", 3: "CC_ERR_HIP",
             4: "CC_ERR_NUMERIC", 5: "CC_ERR_STATE"}
    return names.get(int(s), f"CC_ERR_{int(s)}")


def check(status: int) -> None:
    if status != CC_OK:
        msg = load().cc_last_error_message()
        raise CCError(status, msg.decode() if msg else "")


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load().cc_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o
