"""Cubic Lagrange interpolation on the periodic grid (App. A, Lagrange interpolation).

Around a reduced coordinate t in [0, 1) (the same t and grid index i0 as the B-spline,
Eq. reducedcoordinate) the four grid points l = -1, 0, 1, 2 carry the basis polynomials

    ell_l(t) = prod_{j in {-1, 0, 1, 2}, j != l} (t - j) / (l - j)      (Eq. lagrangebasisgeneral3)

and the tricubic interpolant is the tensor product over the three axes with the grid values
themselves as coefficients (Eq. lagrangeinterpolation3): nothing is solved.  The basis has no
continuous derivative across grid points, so the gradient and the Laplacian are separate
Lagrange interpolants of their own grid values (the paper's direct approximations), not
derivatives of this one.
"""
import numpy as np

from .bspline import OFFSETS
from .evaluate import reduced_coordinates, _block


def weights(t, order=0):
    """ell_l(t) (order 0) or d ell_l / dt (order 1) for l = -1..2, from the product formula
    (the derivative by the product rule: one factor differentiated at a time).
    t: array [...]; returns [..., 4]."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros(t.shape + (4,))
    for a, l in enumerate(OFFSETS):
        others = [j for j in OFFSETS if j != l]
        denom = np.prod([float(l - j) for j in others])
        if order == 0:
            term = np.ones_like(t)
            for j in others:
                term = term * (t - j)
            out[..., a] = term / denom
        elif order == 1:
            for skip in others:
                term = np.ones_like(t)
                for j in others:
                    if j != skip:
                        term = term * (t - j)
                out[..., a] += term / denom
        else:
            raise ValueError("order 0 or 1")
    return out


def eval_values(vals, lattice, pos, chunk=256):
    """Tricubic Lagrange interpolant of grid values vals [N1][N2][N3][O] at pos [P,3]: [P,O].

    Points with non-finite coordinates give NaN.
    """
    vals = np.asarray(vals, dtype=np.float64)
    grid = vals.shape[:3]
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    out = np.empty((i0.shape[0], vals.shape[3]))
    for p0 in range(0, i0.shape[0], chunk):
        sl = slice(p0, p0 + chunk)
        wx, wy, wz = weights(t[sl, 0]), weights(t[sl, 1]), weights(t[sl, 2])
        out[sl] = np.einsum("pl,pm,pn,plmno->po", wx, wy, wz, _block(vals, i0[sl], grid))
    out[~ok] = np.nan
    return out


def eval_abs_bound(vals, lattice, pos, du=None, chunk=256):
    """Rounding-error scales of the interpolant at each point: sum |ell_l ell_m ell_n| |f| (for the
    accumulation error) and, with du [P,3], sum_i du_i sum |d_i(ell ell ell)| |f| (how far a
    perturbation du of the grid coordinates moves the value).  Returns (acc [P,O], coord [P,O])."""
    vals = np.abs(np.asarray(vals, dtype=np.float64))
    grid = vals.shape[:3]
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    n_pts, n_orb = i0.shape[0], vals.shape[3]
    acc = np.zeros((n_pts, n_orb))
    coord = np.zeros((n_pts, n_orb))
    for p0 in range(0, n_pts, chunk):
        sl = slice(p0, p0 + chunk)
        w = [np.abs(weights(t[sl, d])) for d in range(3)]
        dw = [np.abs(weights(t[sl, d], 1)) for d in range(3)]
        blk = _block(vals, i0[sl], grid)
        acc[sl] = np.einsum("pl,pm,pn,plmno->po", w[0], w[1], w[2], blk)
        if du is not None:
            d = np.asarray(du, dtype=np.float64)[sl]
            coord[sl] = (d[:, 0, None] * np.einsum("pl,pm,pn,plmno->po", dw[0], w[1], w[2], blk)
                         + d[:, 1, None] * np.einsum("pl,pm,pn,plmno->po", w[0], dw[1], w[2], blk)
                         + d[:, 2, None] * np.einsum("pl,pm,pn,plmno->po", w[0], w[1], dw[2], blk))
    return acc, coord
