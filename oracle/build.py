"""Interpolating periodic B-spline coefficients (App. A, "Interpolating B-spline coefficients").

The coefficients beta solve

    sum_{l,m,n} B^x_{il} B^y_{jm} B^z_{kn} beta_{lmn} = f_{ijk}    for every grid point (i, j, k),

where B^d_{il} is the value at grid point i of the basis function centred at grid
point l.  With periodic boundary conditions each B^d is tridiagonal with corner
elements.  Because the matrix is a Kronecker product, the system is solved in
three stages, one axis at a time: B^x is applied inversely along the first grid
index for every (j, k, orbital) line, then B^y along the second, then B^z along
the third.

Here every stage is a dense numpy solve with the assembled N x N periodic matrix
(all lines at once as right-hand sides).  Grid values are laid out
[N1][N2][N3][n_orb] (orbital innermost) and the result has the same layout.
"""
import numpy as np

from .bspline import b


def periodic_knot_matrix(n):
    """B[i, l] = value at knot i of the periodic basis function centred at knot l.

    A periodic coefficient sequence means the basis function centred at l is
    also present at l + k n for every integer k, so B[i, l] = sum_k b(i - l - k n).
    For the standard normalization the rows are (1/6, 4/6, 1/6) with corners.
    """
    i = np.arange(n)[:, None].astype(np.float64)
    l = np.arange(n)[None, :].astype(np.float64)
    out = np.zeros((n, n))
    for k in range(-3, 4):
        out += b(i - l - k * n)
    return out


def solve_axis(mat, data, axis):
    """Apply mat^-1 along ``axis`` of ``data`` (every other index is an independent line)."""
    moved = np.moveaxis(data, axis, 0)
    shape = moved.shape
    sol = np.linalg.solve(mat, moved.reshape(shape[0], -1))
    return np.moveaxis(sol.reshape(shape), 0, axis)


def build_interp(values):
    """Coefficients beta [N1][N2][N3][O] of the periodic interpolating tricubic spline of ``values``."""
    values = np.asarray(values, dtype=np.float64)
    if values.ndim == 3:
        values = values[..., None]
    beta = values
    for axis in range(3):
        beta = solve_axis(periodic_knot_matrix(values.shape[axis]), beta, axis)
    return np.ascontiguousarray(beta)
