"""Adjoint of the spline evaluation: gradients of a scalar loss.

The outputs V, grad V and lap V of the evaluation (App. A, Eq. b-splineapproximation,
with the chain rule of Sec. II) are linear in the coefficients beta.  Given the
gradients of a scalar loss L with respect to the outputs, gV [P,O], gG [P,3,O]
and gL [P,O], this module returns

  dL/dbeta[g, o] = sum_p sum_q gq[p, o] * dq[p, o]/dbeta[g, o]
                 (the transpose of the 64-coefficient gather, periodic wrap)
  dL/dr[p]       = sum_o ( gV grad V + gG . Hess V + gL grad(lap V) )[p, o]

where Hess V = J^T H_t J and grad(lap V) = J^T T_t with T_t[k] =
sum_ij M_ij d^3 V / dt_i dt_j dt_k (M = J J^T), using the piecewise-constant
third derivative of the basis.  With a separate Laplacian spline, gL feeds that
spline's coefficients through its value weights and grad(lap V) is the gradient
of that spline.
"""
import numpy as np

from .bspline import OFFSETS
from .evaluate import (jacobian, reduced_coordinates, _block, _weights, _reduced_derivative, _orders)


def _outer(w, orders):
    ox, oy, oz = orders
    return np.einsum("pl,pm,pn->plmn", w[0][ox], w[1][oy], w[2][oz])


def vgl_backward(beta, lattice, pos, gv=None, ggrad=None, glap=None, lap_beta=None, chunk=256):
    """Returns (gbeta [N1,N2,N3,O], glap_beta or None, gpos [P,3])."""
    beta = np.asarray(beta, dtype=np.float64)
    grid = beta.shape[:3]
    n_orb = beta.shape[3]
    jac, metric = jacobian(lattice, grid)
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    n_pts = i0.shape[0]
    zeros_po = np.zeros((n_pts, n_orb))
    gv = zeros_po if gv is None else np.asarray(gv, dtype=np.float64)
    glap = zeros_po if glap is None else np.asarray(glap, dtype=np.float64)
    ggrad = np.zeros((n_pts, 3, n_orb)) if ggrad is None else np.asarray(ggrad, dtype=np.float64)
    lap_b = None if lap_beta is None else np.asarray(lap_beta, dtype=np.float64)

    gbeta = np.zeros_like(beta)
    glap_beta = None if lap_b is None else np.zeros_like(lap_b)
    gpos = np.zeros((n_pts, 3))
    for p0 in range(0, n_pts, chunk):
        sl = slice(p0, p0 + chunk)
        keep = ok[sl]
        w = _weights(t[sl], 3)
        ix = (i0[sl, 0, None] + OFFSETS) % grid[0]
        iy = (i0[sl, 1, None] + OFFSETS) % grid[1]
        iz = (i0[sl, 2, None] + OFFSETS) % grid[2]
        idx = (ix[:, :, None, None], iy[:, None, :, None], iz[:, None, None, :])

        # ---- coefficients: sum of weight tensors times upstream gradients
        wv = _outer(w, (0, 0, 0))                                                # [p,4,4,4]
        wt = [_outer(w, _orders(i)) for i in range(3)]                           # d/dt_i
        contrib = np.einsum("plmn,po->plmno", wv, gv[sl])
        for alpha in range(3):
            w_alpha = sum(jac[i, alpha] * wt[i] for i in range(3))               # d/dr_alpha
            contrib += np.einsum("plmn,po->plmno", w_alpha, ggrad[sl, alpha])
        if lap_b is None:
            w_lap = sum(metric[i, j] * _outer(w, _orders(i, j)) for i in range(3) for j in range(3))
            contrib += np.einsum("plmn,po->plmno", w_lap, glap[sl])
        else:
            lcontrib = np.einsum("plmn,po->plmno", wv, glap[sl])
            lcontrib[~keep] = 0.0
            np.add.at(glap_beta, idx, lcontrib)
        contrib[~keep] = 0.0
        np.add.at(gbeta, idx, contrib)

        # ---- positions
        blk = _block(beta, i0[sl], grid)
        g_t = np.stack([_reduced_derivative(blk, w, _orders(i)) for i in range(3)], axis=1)       # [p,3,O]
        h_t = np.empty((blk.shape[0], 3, 3, n_orb))
        for i in range(3):
            for j in range(3):
                h_t[:, i, j] = _reduced_derivative(blk, w, _orders(i, j))
        if lap_b is None:
            third = np.zeros((blk.shape[0], 3, n_orb))
            for k in range(3):
                for i in range(3):
                    for j in range(3):
                        third[:, k] += metric[i, j] * _reduced_derivative(blk, w, _orders(i, j, k))
        else:
            lblk = _block(lap_b, i0[sl], grid)
            third = np.stack([_reduced_derivative(lblk, w, _orders(k)) for k in range(3)], axis=1)
        grad_cart = np.einsum("ia,pio->pao", jac, g_t)                          # grad V
        hess_cart = np.einsum("ia,jb,pijo->pabo", jac, jac, h_t)                # Hess V
        glap_cart = np.einsum("ka,pko->pao", jac, third)                        # grad lap V
        gp = (np.einsum("po,pao->pa", gv[sl], grad_cart)
              + np.einsum("pbo,pbao->pa", ggrad[sl], hess_cart)
              + np.einsum("po,pao->pa", glap[sl], glap_cart))
        gp[~keep] = np.nan
        gpos[sl] = gp
    return gbeta, glap_beta, gpos
