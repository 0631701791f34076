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


def weights(t):
    """ell_l(t) for l = -1..2, from the product formula.  t: array [...]; returns [..., 4]."""
    t = np.asarray(t, dtype=np.float64)
    out = np.ones(t.shape + (4,))
    for a, l in enumerate(OFFSETS):
        for j in OFFSETS:
            if j != l:
                out[..., a] *= (t - j) / (l - j)
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
