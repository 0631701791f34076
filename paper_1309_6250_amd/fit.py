"""Least-squares fit of spline coefficients to planewave orbital data, driven by the adjoint.

Minimizes over the coefficient table beta (FP32 or FP64)

  L = wV mean (V - V_t)^2 + wL mean (lap - lap_t)^2
      + lam * sum over orbitals, axes and grid points of (second difference of beta)^2
            / (N1 N2 N3 n_orb mean V_t^2)

with wV = 1 / mean V_t^2 and wL = 1 / mean lap_t^2 (or 0), periodic second differences,
by Adam.  V and lap come from the library's forward kernel and the gradient of the misfit
terms from its adjoint kernel (SplineVGL); the penalty, the reductions and the Adam update
are small elementwise tensor operations on the table.  The residuals are formed in the
kernel's output precision (FP64 for FP64 tables, FP32 otherwise) and their squares summed in
FP64.
"""
import torch

from ._lib import SPL_DETERMINISTIC
from .api import OUT_TORCH
from .autograd import SplineVGL


def second_difference(beta, dim):
    return torch.roll(beta, 1, dims=dim) - 2.0 * beta + torch.roll(beta, -1, dims=dim)


def make_loss(desc, pos, v_t, lap_t, lam=1e-3, use_lap=True, deterministic=True, sorted_forward=True):
    n_orb = desc.n_orb
    v64 = v_t.to(torch.float64)
    l64 = lap_t.to(torch.float64)
    w_v = 1.0 / torch.mean(v64 * v64)
    w_l = (1.0 / torch.mean(l64 * l64)) if use_lap else torch.zeros((), dtype=torch.float64, device=v_t.device)
    pts = desc.grid[0] * desc.grid[1] * desc.grid[2]
    reg_scale = lam / (pts * n_orb * torch.mean(v64 * v64))
    od = OUT_TORCH[desc.dtype]
    v_t = v_t.to(od).contiguous()
    lap_t = lap_t.to(od).contiguous()
    del v64, l64

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


def fit_adam(desc, table, pos, v_t, lap_t, steps=200, lam=1e-3, lr=None, use_lap=True, callback=None,
             deterministic=True, sorted_forward=True):
    """Adam from `table` (not modified); returns (fitted table, list of losses per step).
    deterministic: bitwise-reproducible coefficient gradients (cell-sorted accumulation);
    sorted_forward: forward evaluation in locality order (same outputs)."""
    beta = table.detach().clone().requires_grad_(True)
    loss_fn = make_loss(desc, pos, v_t, lap_t, lam=lam, use_lap=use_lap, deterministic=deterministic,
                        sorted_forward=sorted_forward)
    if lr is None:
        lr = 1e-3 * float(torch.sqrt(torch.mean(table.detach().to(torch.float64) ** 2)))
    opt = torch.optim.Adam([beta], lr=lr, betas=(0.9, 0.999))
    losses = []
    for step in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = loss_fn(beta)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
        if callback is not None:
            callback(step, losses[-1])
    return beta.detach(), losses
