"""torch.autograd binding of the forward VGL kernel and its adjoint.

SplineVGL.apply(table, pos, desc) -> (v, grad, lap), differentiable with respect to the
coefficient table and the positions.  Both directions run in the library's kernels
(spline_eval_vgl and spline_eval_vgl_backward); this module only passes tensors.

For BF16 tables the coefficient gradient is produced in FP32 and autograd casts it to the
table's dtype; keep FP32 master coefficients when training.
"""
import torch

from ._lib import SPL_DETERMINISTIC
from .api import spline_eval_vgl, spline_eval_vgl_sorted, spline_eval_vgl_backward, OUT_TORCH


class SplineVGL(torch.autograd.Function):
    """Outputs a loss does not use get no gradient tensor (None reaches the adjoint as NULL, so
    that term is skipped instead of read as zeros).  flags: SPL_DETERMINISTIC (the default: the
    cell-sorted adjoint, bitwise reproducible and also the faster one, at every point density
    measured) or 0 (float atomics).  sorted_forward runs the forward through
    spline_eval_vgl_sorted (the same outputs, bitwise, evaluated in locality order)."""

    @staticmethod
    def forward(ctx, table, pos, desc, flags=SPL_DETERMINISTIC, sorted_forward=False):
        ctx.set_materialize_grads(False)
        if sorted_forward:
            v, g, l = spline_eval_vgl_sorted(desc, table, pos)
        else:
            v, g, l = spline_eval_vgl(desc, table, pos)
        ctx.save_for_backward(table, pos)
        ctx.desc = desc
        ctx.flags = flags
        return v, g, l

    @staticmethod
    def backward(ctx, gv, gg, gl):
        table, pos = ctx.saved_tensors
        desc = ctx.desc
        od = OUT_TORCH[desc.dtype]
        prep = [None if g is None else g.to(od).contiguous() for g in (gv, gg, gl)]
        want_t, want_p = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_t or want_p):
            return None, None, None, None, None
        gtable, gpos = spline_eval_vgl_backward(desc, table, pos, *prep, want_table=want_t, want_pos=want_p,
                                                flags=ctx.flags)
        return gtable, gpos, None, None, None


def spline_vgl(table, pos, desc, deterministic=True, sorted_forward=False):
    """Differentiable (v, grad, lap) of the spline `table` at `pos`.  deterministic=True (default):
    the coefficient gradient is accumulated cell by cell, bitwise reproducible; False: float
    atomics.  sorted_forward=True evaluates the points in locality order (same outputs)."""
    return SplineVGL.apply(table, pos, desc, SPL_DETERMINISTIC if deterministic else 0, sorted_forward)
