"""Periodic tricubic B-spline orbital evaluation on AMD Instinct MI355X (gfx950).

The computation lives in the HIP library libpwspline.so (C ABI in
include/pwspline.h); this package only binds it.  Importing the package does not
load the library; the first call does, and fails loudly if it was not built.
"""
from ._lib import (SPL_F64, SPL_F32, SPL_BF16, SPL_OK, SPL_EINVAL, SPL_EGRID, SPL_EDTYPE, SPL_ENOMEM, SPL_EHIP,
                   SPL_EUNSUPPORTED, SPL_DETERMINISTIC, SPL_REUSE_SORT, SPL_BSPLINE, SPL_LAGRANGE, SPL_PPSPLINE, SplineError, SplDesc, EXPORTS,
                   LIB_PATH, lib)
from .api import (spline_desc_init, spline_build, spline_build_tables, spline_eval_v, spline_eval_vgl,
                  spline_eval_vgl_sorted, spline_sorted_work_bytes, spline_eval_vgl_sorted_noalloc, spline_eval_vgl_cells,
                  spline_cells_work_bytes, spline_fit_terms_cells, spline_fit_gradient_cells,
                  spline_fit_gradient_work_bytes, spline_adam_step,
                  spline_eval_vgl_backward,
                  spline_autotune, spline_tile_for, spline_backward_work_bytes, spline_build_smoothing,
                  spline_smoothing_work_bytes, spline_misfit, spline_misfit_work_bytes, spline_smoothness_penalty,
                  spline_stream_read, BatchPlan, new_table,
                  new_gtable, table_shape,
                  STORE_TORCH, OUT_TORCH, DTYPES)
from .autograd import SplineVGL, spline_vgl

__all__ = [
    "spline_desc_init", "spline_build", "spline_build_tables", "spline_eval_v", "spline_eval_vgl_sorted",
    "spline_eval_vgl_cells", "spline_cells_work_bytes", "spline_fit_terms_cells", "spline_fit_gradient_cells",
    "spline_fit_gradient_work_bytes", "spline_adam_step", "spline_eval_vgl_sorted_noalloc",
    "spline_sorted_work_bytes", "spline_eval_vgl", "spline_eval_vgl_backward",
    "spline_autotune", "spline_tile_for", "spline_backward_work_bytes", "spline_build_smoothing",
    "spline_smoothing_work_bytes", "spline_misfit", "spline_misfit_work_bytes", "spline_smoothness_penalty",
    "spline_stream_read", "BatchPlan", "new_table", "new_gtable", "table_shape", "SplineError",
    "SplDesc", "lib", "EXPORTS", "LIB_PATH", "SPL_F64", "SPL_F32", "SPL_BF16", "SPL_OK", "SPL_EINVAL", "SPL_EGRID",
    "SPL_EDTYPE", "SPL_ENOMEM", "SPL_EHIP", "SPL_EUNSUPPORTED", "SPL_DETERMINISTIC", "SPL_REUSE_SORT", "SPL_BSPLINE", "SPL_LAGRANGE", "SPL_PPSPLINE", "STORE_TORCH", "OUT_TORCH",
    "DTYPES", "SplineVGL", "spline_vgl",
]
