"""ctypes view of libpwspline.so (the C ABI declared in include/pwspline.h).

Loading fails loudly when the library has not been built: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwspline.so")

SPL_F64, SPL_F32, SPL_BF16 = 0, 1, 2
SPL_OK, SPL_EINVAL, SPL_EGRID, SPL_EDTYPE, SPL_ENOMEM, SPL_EHIP, SPL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SPL_DETERMINISTIC = 1
SPL_REUSE_SORT = 2
SPL_BSPLINE, SPL_LAGRANGE, SPL_PPSPLINE = 0, 1, 2

ERROR_NAMES = {
    SPL_EINVAL: "SPL_EINVAL", SPL_EGRID: "SPL_EGRID", SPL_EDTYPE: "SPL_EDTYPE", SPL_ENOMEM: "SPL_ENOMEM",
    SPL_EHIP: "SPL_EHIP", SPL_EUNSUPPORTED: "SPL_EUNSUPPORTED",
}

EXPORTS = (
    "spline_desc_init", "spline_build", "spline_eval_v", "spline_eval_vgl", "spline_eval_vgl_tile",
    "spline_eval_vgl_backward", "spline_batch_plan_create", "spline_batch_eval_vgl",
    "spline_batch_graph_launch", "spline_batch_autotune", "spline_batch_plan_destroy", "spline_batch_plan_info", "spline_autotune",
    "spline_tile_for", "spline_last_error", "spline_version", "spline_backward_work_bytes",
    "spline_build_smoothing", "spline_smoothing_work_bytes", "spline_build_tables",
    "spline_eval_vgl_sorted", "spline_sorted_work_bytes", "spline_batch_plan_sort", "spline_misfit",
    "spline_misfit_work_bytes", "spline_smoothness_penalty", "spline_eval_vgl_cells", "spline_cells_work_bytes",
    "spline_fit_terms_cells", "spline_stream_read", "spline_eval_vgl_sorted_noalloc",
    "spline_batch_plan_get_tiles", "spline_batch_plan_set_tiles", "spline_fit_gradient_cells",
    "spline_fit_gradient_work_bytes", "spline_adam_step",
)


class SplDesc(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_double * 9),
        ("grid", ctypes.c_int32 * 3),
        ("n_orb", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("has_lap", ctypes.c_int32),
        ("basis", ctypes.c_int32),
        ("sep_grad", ctypes.c_int32),
        ("bloch", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("kvec", ctypes.c_double * 3),
        ("ainv", ctypes.c_double * 9),
        ("jac", ctypes.c_double * 9),
        ("metric", ctypes.c_double * 6),
        ("o_pad", ctypes.c_int32),
        ("elem_bytes", ctypes.c_int32),
        ("table_elems", ctypes.c_int64),
        ("table_bytes", ctypes.c_int64),
        ("work_bytes", ctypes.c_int64),
        ("gtable_bytes", ctypes.c_int64),
        ("n_tables", ctypes.c_int32),
        ("n_col", ctypes.c_int32),
    ]


class SplItem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.POINTER(SplDesc)),
        ("table", ctypes.c_void_p),
        ("n_pts", ctypes.c_int64),
        ("pos", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("grad", ctypes.c_void_p),
        ("lap", ctypes.c_void_p),
    ]


class SplineError(RuntimeError):
    def __init__(self, code, func, message):
        super().__init__(f"{func} failed with {ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


_lib = None


def lib():
    """The loaded library (loads it on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1309_6250_amd.build_lib "
                              "(or __graft_entry__.build())")
        h = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        pd = ctypes.POINTER(SplDesc)
        i32p = ctypes.POINTER(ctypes.c_int32)
        sig = {
            "spline_desc_init": (ctypes.c_int, [pd]),
            "spline_build": (ctypes.c_int, [pd, vp, vp, vp, vp, vp]),
            "spline_build_tables": (ctypes.c_int, [pd, vp, vp, vp, vp]),
            "spline_eval_vgl_sorted": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, i32p, vp, i64, vp]),
            "spline_sorted_work_bytes": (ctypes.c_int, [pd, i64, ctypes.POINTER(i64)]),
            "spline_eval_vgl_sorted_noalloc": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, i32p, vp]),
            "spline_eval_v": (ctypes.c_int, [pd, vp, i64, vp, vp, vp]),
            "spline_eval_vgl": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, vp]),
            "spline_eval_vgl_tile": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, i32p, vp]),
            "spline_eval_vgl_backward": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, vp, vp, i32, vp, i64, vp]),
            "spline_backward_work_bytes": (ctypes.c_int, [pd, i64, i32, ctypes.POINTER(i64)]),
            "spline_misfit": (ctypes.c_int, [pd, i64, vp, vp, ctypes.c_double, vp, vp, vp, i64, vp]),
            "spline_misfit_work_bytes": (ctypes.c_int, [pd, i64, ctypes.POINTER(i64)]),
            "spline_smoothness_penalty": (ctypes.c_int, [pd, vp, ctypes.c_double, vp, vp, vp, i64, vp]),
            "spline_eval_vgl_cells": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, i32, vp, i64, vp]),
            "spline_cells_work_bytes": (ctypes.c_int, [pd, i64, ctypes.POINTER(i64)]),
            "spline_fit_terms_cells": (ctypes.c_int, [pd, vp, i64, vp, vp, ctypes.c_double, vp, vp, ctypes.c_double,
                                                      vp, vp, i32, vp, i64, vp]),
            "spline_fit_gradient_cells": (ctypes.c_int, [pd, vp, i64, vp, vp, ctypes.c_double, vp, ctypes.c_double,
                                                         vp, vp, i32, vp, i64, vp]),
            "spline_fit_gradient_work_bytes": (ctypes.c_int, [pd, i64, ctypes.POINTER(i64)]),
            "spline_adam_step": (ctypes.c_int, [i32, i64, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, i32, vp]),
            "spline_build_smoothing": (ctypes.c_int, [pd, i64, vp, vp, vp, vp, vp]),
            "spline_smoothing_work_bytes": (ctypes.c_int, [pd, ctypes.POINTER(i64)]),
            "spline_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(SplItem), i32, i32p, vp,
                                                        ctypes.POINTER(vp)]),
            "spline_batch_eval_vgl": (ctypes.c_int, [vp, vp]),
            "spline_batch_graph_launch": (ctypes.c_int, [vp, vp]),
            "spline_batch_autotune": (ctypes.c_int, [vp, vp, i32p]),
            "spline_batch_plan_destroy": (None, [vp]),
            "spline_batch_plan_sort": (ctypes.c_int, [vp, i32, vp]),
            "spline_batch_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
            "spline_batch_plan_get_tiles": (ctypes.c_int, [vp, i32p]),
            "spline_batch_plan_set_tiles": (ctypes.c_int, [vp, i32p, vp]),
            "spline_autotune": (ctypes.c_int, [pd, vp, i64, vp, vp, vp, vp, vp, i32p]),
            "spline_tile_for": (ctypes.c_int, [pd, i64, i32p]),
            "spline_stream_read": (ctypes.c_int, [vp, i64, vp, vp]),
            "spline_last_error": (ctypes.c_char_p, []),
            "spline_version": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(code, func):
    if code != SPL_OK:
        msg = lib().spline_last_error().decode(errors="replace")
        raise SplineError(code, func, msg)
    return code
