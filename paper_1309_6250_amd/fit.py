"""Least-squares fit of spline coefficients to planewave orbital data, driven by the adjoint.

Minimizes over the coefficient table beta (FP32 or FP64)

  L = wV mean (V - V_t)^2 + wL mean (lap - lap_t)^2
      + lam * sum over orbitals, axes and grid points of (second difference of beta)^2
            / (N1 N2 N3 n_orb mean V_t^2)

with wV = 1 / mean V_t^2 and wL = 1 / mean lap_t^2 (or 0), periodic second differences,
by Adam.  Two forms of the same loss:

- FitProblem.loss_and_grad and FitProblem.adam_step, used by fit_adam: every term runs in the
  library's kernels (spline_fit_terms_cells, the cell-wise forward of V and lap that forms the
  upstream gradients 2 w (y - t) as it evaluates and sums the squared residuals in FP64 in a fixed
  order; the adjoint; spline_smoothness_penalty on the table), and so does the Adam update
  (spline_adam_step).  Buffers are allocated once.  With fused=False the forward writes V and lap and
  spline_misfit forms the same gradients from them in a second pass.
- make_loss, a differentiable function of the table built on SplineVGL, for use inside a
  larger autograd graph.  Its residuals are formed in the kernel's output precision and
  their squares summed in FP64.
"""
import math

import torch

from ._lib import SPL_DETERMINISTIC, SPL_F32, SPL_REUSE_SORT
from .api import (OUT_TORCH, new_gtable, spline_adam_step, spline_eval_vgl_backward, spline_eval_vgl_cells,
                  spline_fit_terms_cells, spline_fit_gradient_cells,
                  spline_fit_gradient_work_bytes,
                  spline_misfit, spline_misfit_work_bytes, spline_smoothness_penalty, spline_cells_work_bytes,
                  spline_backward_work_bytes)
from .autograd import SplineVGL


def second_difference(beta, dim):
    return torch.roll(beta, 1, dims=dim) - 2.0 * beta + torch.roll(beta, -1, dims=dim)


def _weights(desc, v_t, lap_t, lam, use_lap):
    v64 = v_t.to(torch.float64)
    mv = torch.mean(v64 * v64)
    w_v = 1.0 / mv
    if use_lap:
        l64 = lap_t.to(torch.float64)
        w_l = 1.0 / torch.mean(l64 * l64)
    else:
        w_l = torch.zeros((), dtype=torch.float64, device=v_t.device)
    pts = desc.grid[0] * desc.grid[1] * desc.grid[2]
    reg_scale = lam / (pts * desc.n_orb * mv)
    return w_v, w_l, reg_scale


def make_loss(desc, pos, v_t, lap_t, lam=1e-3, use_lap=True, deterministic=True, sorted_forward=True):
    n_orb = desc.n_orb
    w_v, w_l, reg_scale = _weights(desc, v_t, lap_t, lam, use_lap)
    od = OUT_TORCH[desc.dtype]
    v_t = v_t.to(od).contiguous()
    lap_t = lap_t.to(od).contiguous()

    flags = SPL_DETERMINISTIC if deterministic else 0

    def loss_fn(beta):
        v, _, lap = SplineVGL.apply(beta, pos, desc, flags, sorted_forward)
        rv = v - v_t
        loss = w_v * torch.mean(rv * rv, dtype=torch.float64)
        if use_lap:
            rl = lap - lap_t
            loss = loss + w_l * torch.mean(rl * rl, dtype=torch.float64)
        if lam:
            core = beta[0, ..., :n_orb].to(torch.float64)      # orbital table, real orbitals only
            reg = sum(torch.sum(second_difference(core, d) ** 2) for d in range(3))
            loss = loss + reg_scale * reg
        return loss

    return loss_fn


class FitProblem:
    """The fit's loss and its coefficient gradient at fixed points pos [P][3] with targets
    v_t, lap_t [P][n_orb], without autograd.  loss_and_grad(beta) returns (loss, grad) as
    device tensors (FP64 scalar; the gradient table, FP32 for FP32 and BF16 tables); both are
    reused by the next call.

    fused: the misfit is formed inside the cell-wise forward; where spline_fit_gradient_cells
    applies (FP32 table, Laplacian from derivatives, both terms, deterministic, at least 4 points per
    cell, table and targets under 2 GiB) the forward, the misfit and the adjoint run as one pass,
    with the same bits.  Otherwise, or with fused=False, the forward and spline_misfit write the
    residual gradients, which the adjoint then reads."""

    def __init__(self, desc, pos, v_t, lap_t, lam=1e-3, use_lap=True, deterministic=True, fused=True):
        self.desc, self.pos, self.lam, self.use_lap, self.fused = desc, pos, lam, use_lap, fused
        self.flags = SPL_DETERMINISTIC if deterministic else 0
        w_v, w_l, reg_scale = _weights(desc, v_t, lap_t, lam, use_lap)
        n, o = pos.shape[0], desc.n_orb
        self.w_v, self.w_l = float(w_v) / (n * o), float(w_l) / (n * o)
        self.reg_scale = float(reg_scale)
        od = OUT_TORCH[desc.dtype]
        dev = pos.device
        self.v_t = v_t.to(od).contiguous()
        self.lap_t = lap_t.to(od).contiguous()
        self.v = torch.empty((n, o), dtype=od, device=dev)
        self.lap = torch.empty((n, o), dtype=od, device=dev)
        self.gtable = new_gtable(desc, dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        # one workspace for the forward and the adjoint: the points never move, so the cell sort
        # made by the first forward serves every later call (SPL_REUSE_SORT)
        self.misfit_work = torch.empty(spline_misfit_work_bytes(desc, n * o), dtype=torch.uint8, device=dev)
        self.reuse = deterministic
        cells = desc.grid[0] * desc.grid[1] * desc.grid[2]
        under = (1 << 31) - 4096
        self.one_pass = (fused and deterministic and use_lap and desc.dtype == SPL_F32 and not desc.has_lap
                         and 2 * n >= 5 * cells and desc.table_bytes < under and 4 * n * o < under)
        nb = max(spline_cells_work_bytes(desc, n), spline_backward_work_bytes(desc, n, self.flags))
        if self.one_pass:
            nb = max(nb, spline_fit_gradient_work_bytes(desc, n))
        self.work = torch.empty(max(1, nb), dtype=torch.uint8, device=dev)
        self.sorted = False

    def loss_and_grad(self, beta):
        d = self.desc
        self.loss.zero_()
        reuse = SPL_REUSE_SORT if self.sorted else 0
        lap = self.lap if self.use_lap else None
        if self.one_pass:
            # forward, misfit and adjoint of every batch of points in one kernel
            self.gtable.zero_()
            spline_fit_gradient_cells(d, beta, self.pos, self.v_t, self.w_v, self.lap_t, self.w_l, gtable=self.gtable,
                                      loss=self.loss, work=self.work, flags=reuse)
            self.sorted = True
            if self.lam:
                spline_smoothness_penalty(d, beta, self.reg_scale, self.loss, gtable=self.gtable,
                                          work=self.misfit_work)
            return self.loss, self.gtable
        if self.fused:
            # the residuals and their sum straight from the cell-wise evaluation
            gv, gl, _ = spline_fit_terms_cells(d, beta, self.pos, self.v_t, self.w_v,
                                               self.lap_t if self.use_lap else None, self.w_l, g_v=self.v,
                                               g_lap=lap, loss=self.loss, work=self.work, flags=reuse)
        else:
            spline_eval_vgl_cells(d, beta, self.pos, self.v, None, lap, outputs="vl" if self.use_lap else "v",
                                  work=self.work, flags=reuse)
            gv = spline_misfit(d, self.v, self.v_t, self.w_v, self.loss, g=self.v, work=self.misfit_work)
            gl = None
            if self.use_lap:
                gl = spline_misfit(d, self.lap, self.lap_t, self.w_l, self.loss, g=self.lap, work=self.misfit_work)
        self.sorted = self.reuse
        self.gtable.zero_()
        spline_eval_vgl_backward(d, beta, self.pos, gv, None, gl, self.gtable, None, want_pos=False,
                                 flags=self.flags | (SPL_REUSE_SORT if self.sorted else 0),
                                 work=self.work if self.flags else None)
        if self.lam:
            spline_smoothness_penalty(d, beta, self.reg_scale, self.loss, gtable=self.gtable, work=self.misfit_work)
        return self.loss, self.gtable

    def adam_step(self, beta, m, v, lr, step, betas=(0.9, 0.999), eps=1e-8):
        """One Adam step (Kingma and Ba, Algorithm 1; `step` counts from 1) on the loss at `beta`: the
        table is updated in place by spline_adam_step from the gradient of loss_and_grad, the moments
        m and v (FP64 for FP64 tables, else FP32) likewise, and the loss at the old `beta` is returned
        (a one-element FP64 device tensor, reused by the next call)."""
        loss, g = self.loss_and_grad(beta)
        spline_adam_step(beta, g, m, v, lr, step, beta1=betas[0], beta2=betas[1], eps=eps)
        return loss


def fit_adam(desc, table, pos, v_t, lap_t, steps=200, lam=1e-3, lr=None, use_lap=True, callback=None,
             deterministic=True, checkpoint=None, checkpoint_every=0, schedule="cosine", lr_min_frac=0.01):
    """Adam from `table` (not modified); returns (fitted table, list of losses of every step run so
    far, including those before a resume).
    lr: the step size (default 0.1 rms(table): on the 64-atom fit workload 200 steps from the
    interpolating spline then reach the loss of the exact optimum, where 1e-3 rms closes a few per
    cent of that gap); schedule "constant", or "cosine" (default): step k of `steps` uses
    lr_min + (lr - lr_min)(1 + cos(pi k / steps)) / 2 with lr_min = lr_min_frac lr (a function of k
    alone, so a resumed fit takes the same steps).
    deterministic: bitwise-reproducible coefficient gradients (cell-sorted accumulation).
    checkpoint: file path.  If it exists, the fit resumes from it (coefficients, Adam moments m and v
    and step count, loaded with torch.load(weights_only=True)); every `checkpoint_every` steps (and
    after the last step) the state is written there, to a temporary file first and then renamed.
    With the deterministic gradient a resumed fit retraces the uninterrupted one bit for bit."""
    import os
    prob = FitProblem(desc, pos, v_t, lap_t, lam=lam, use_lap=use_lap, deterministic=deterministic)
    beta = table.detach().clone()
    mom = torch.float64 if beta.dtype == torch.float64 else torch.float32
    m = torch.zeros(beta.shape, dtype=mom, device=beta.device)
    v = torch.zeros_like(m)
    if lr is None:
        lr = 0.1 * float(torch.sqrt(torch.mean(table.detach().to(torch.float64) ** 2)))
    start, done = 0, []
    if checkpoint is not None and os.path.exists(checkpoint):
        state = torch.load(checkpoint, map_location=beta.device, weights_only=True)
        if tuple(state["beta"].shape) != tuple(beta.shape) or state["beta"].dtype != beta.dtype:
            raise ValueError(f"{checkpoint} holds a table of another shape or dtype")
        beta.copy_(state["beta"])
        m.copy_(state["m"])
        v.copy_(state["v"])
        start, done = int(state["step"]), [float(x) for x in state["losses"]]

    def save(step, losses):
        tmp = checkpoint + ".tmp"
        torch.save({"beta": beta, "m": m, "v": v, "step": step,
                    "losses": torch.tensor(done + [float(x) for x in torch.cat(losses).cpu()] if losses else done,
                                           dtype=torch.float64)}, tmp)
        os.replace(tmp, checkpoint)

    if schedule not in ("constant", "cosine"):
        raise ValueError(f"unknown schedule {schedule!r}")
    lr_min = lr_min_frac * lr
    losses = []
    for step in range(start, steps):
        lr_k = lr
        if schedule == "cosine":
            lr_k = lr_min + (lr - lr_min) * 0.5 * (1.0 + math.cos(math.pi * step / steps))
        loss = prob.adam_step(beta, m, v, lr_k, step + 1)
        losses.append(loss.clone())
        if callback is not None:
            callback(step, float(losses[-1]))
        if checkpoint is not None and (step + 1 == steps or (checkpoint_every and (step + 1) % checkpoint_every == 0)):
            save(step + 1, losses)
    return beta.detach(), done + ([float(x) for x in torch.cat(losses).cpu()] if losses else [])


def fit_optimum_cg(desc, table, pos, v_t, lap_t, lam=1e-3, use_lap=True, iters=300, rtol=1e-9):
    """The minimizer of the fit loss, by conjugate gradients from `table`.  The loss is a quadratic
    in the coefficients, L(beta) = beta^T H beta / 2 - b^T beta + c, so its gradient g(beta) = H beta - b
    is linear and H p = g(p) - g(0): one gradient per iteration (the library's fit terms, adjoint and
    penalty kernels).  Stops when the residual norm falls below rtol times its first value.  Returns
    (beta, loss at beta, iterations run, relative residual)."""
    if table.dtype not in (torch.float32, torch.float64):
        raise ValueError("conjugate gradients need an FP32 or FP64 table (H p must be formed from p exactly)")
    prob = FitProblem(desc, pos, v_t, lap_t, lam=lam, use_lap=use_lap, deterministic=True)
    x = table.detach().clone()
    _, g = prob.loss_and_grad(torch.zeros_like(x))
    b = -g.clone()
    _, g = prob.loss_and_grad(x)
    r = -g.clone()
    p = r.clone()
    rs = torch.sum(r.double() * r.double())
    rs0 = float(rs)
    it = 0
    for it in range(1, iters + 1):
        _, gp = prob.loss_and_grad(p)
        hp = gp + b
        alpha = rs / torch.sum(p.double() * hp.double())
        x += alpha.to(x.dtype) * p
        r -= alpha.to(r.dtype) * hp
        rs_new = torch.sum(r.double() * r.double())
        if float(rs_new) <= rtol * rtol * rs0:
            rs = rs_new
            break
        p = r + (rs_new / rs).to(r.dtype) * p
        rs = rs_new
    loss, _ = prob.loss_and_grad(x)
    return x, float(loss), it, math.sqrt(float(rs) / rs0) if rs0 > 0 else 0.0
