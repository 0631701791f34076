"""Least-squares fit of spline coefficients to planewave orbital data.

The paper's smoothing spline is a Fourier-matched construction (App. A,
Eq. b-splinecoefficients).  The fit here is its regression counterpart, used
to exercise the adjoint: minimize over beta

  L(beta) = wV mean_{p,o} (V - V_PW)^2 + wL mean_{p,o} (lap - lap_PW)^2
            + lam * sum_o sum_axes sum_grid (beta_{i-1} - 2 beta_i + beta_{i+1})^2
                  / (N1 N2 N3 O mean V_PW^2)

with wV = 1 / mean V_PW^2, wL = 1 / mean lap_PW^2 (or 0), second differences
periodic along each grid axis.  V and lap are the spline's value and
derivative-Laplacian at fixed points.
"""
import numpy as np

from .evaluate import eval_vgl
from .adjoint import vgl_backward


def second_difference(beta, axis):
    return np.roll(beta, 1, axis=axis) - 2.0 * beta + np.roll(beta, -1, axis=axis)


def loss_and_grad(beta, lattice, pos, v_pw, lap_pw, w_v, w_l, lam, want_grad=True):
    """Returns (loss, dloss/dbeta); the gradient is None when want_grad is False."""
    beta = np.asarray(beta, dtype=np.float64)
    n_pts, n_orb = v_pw.shape
    v, _, lap = eval_vgl(beta, lattice, pos)
    norm = 1.0 / (n_pts * n_orb)
    rv = v - v_pw
    rl = lap - lap_pw
    loss = w_v * norm * np.sum(rv * rv) + w_l * norm * np.sum(rl * rl)
    gv = 2.0 * w_v * norm * rv
    gl = 2.0 * w_l * norm * rl
    gbeta = vgl_backward(beta, lattice, pos, gv=gv, glap=gl)[0] if want_grad else None
    if lam:
        scale = lam / (beta[..., 0].size * n_orb * np.mean(v_pw * v_pw))
        reg = 0.0
        for axis in range(3):
            d2 = second_difference(beta, axis)
            reg += np.sum(d2 * d2)
            # d/dbeta sum (D2 beta)^2 = 2 D2^T D2 beta, and D2 is symmetric under periodic wrap
            if want_grad:
                gbeta = gbeta + 2.0 * scale * second_difference(d2, axis)
        loss += scale * reg
    return loss, gbeta


def weights_from_targets(v_pw, lap_pw, use_lap=True):
    w_v = 1.0 / np.mean(v_pw * v_pw)
    w_l = (1.0 / np.mean(lap_pw * lap_pw)) if use_lap else 0.0
    return w_v, w_l
