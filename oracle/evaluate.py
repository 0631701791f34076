"""Tensor-product B-spline evaluation with the chain rule (Sec. II Coordinates; App. A, Eq. b-splineapproximation).

For a Cartesian point r:
  1. crystal coordinates s = a^-1 r, with a the matrix whose columns are the
     lattice vectors (here a = lattice.T);
  2. fold into the cell: s - floor(s);
  3. grid units u_i = N_i (s_i - floor(s_i)); grid index i0 = floor(u_i) and the
     reduced coordinate t_i = u_i - i0 in [0, 1) (Eq. reducedcoordinate);
  4. phi = sum_{l,m,n=-1..2} b_l(t_x) b_m(t_y) b_n(t_z) beta[i0x+l, i0y+m, i0z+n]
     with grid indices taken modulo N (periodic table);
  5. chain rule: with J[i, alpha] = N_i (a^-1)[i, alpha] = d u_i / d r_alpha,
     grad phi = J^T grad_t phi and lap phi = sum_ij (J J^T)_ij d^2 phi / dt_i dt_j.
     The off-diagonal terms matter for non-orthogonal cells.

Step 5's reading: the paper prints N_grid,i outside the transform and
N_grid,i^2 outside the double sum; the grid sizes belong inside, per axis, as in
J above (they differ when the N_i differ).

A point whose coordinates are not finite gets NaN outputs.
"""
import numpy as np

from .bspline import weights, OFFSETS


def jacobian(lattice, grid):
    """J[i, alpha] = N_i (a^-1)[i, alpha] and the metric M = J J^T."""
    a = np.asarray(lattice, dtype=np.float64).T
    jac = np.asarray(grid, dtype=np.float64)[:, None] * np.linalg.inv(a)
    return jac, jac @ jac.T


def reduced_coordinates(lattice, grid, pos):
    """Grid index i0 [P,3] (int64, in [0, N)) and reduced coordinate t [P,3] in [0, 1).

    Also returns a mask of points with finite coordinates; others get i0 = 0, t = 0.
    """
    a = np.asarray(lattice, dtype=np.float64).T
    pos = np.asarray(pos, dtype=np.float64)
    ok = np.all(np.isfinite(pos), axis=1)
    safe = np.where(ok[:, None], pos, 0.0)
    s = np.linalg.solve(a, safe.T).T                   # crystal coordinates
    ok &= np.all(np.isfinite(s), axis=1)                # finite positions can still overflow here
    s = np.where(ok[:, None], s, 0.0)
    frac = s - np.floor(s)
    n = np.asarray(grid, dtype=np.float64)
    u = n * frac
    i0 = np.floor(u)
    t = u - i0
    i0 = i0.astype(np.int64)
    wrap = i0 >= np.asarray(grid)                       # frac or u rounded up to the cell edge
    i0 = np.where(wrap, i0 - np.asarray(grid), i0)
    return i0, t, ok


def _block(beta, i0, grid):
    ix = (i0[:, 0, None] + OFFSETS) % grid[0]
    iy = (i0[:, 1, None] + OFFSETS) % grid[1]
    iz = (i0[:, 2, None] + OFFSETS) % grid[2]
    return beta[ix[:, :, None, None], iy[:, None, :, None], iz[:, None, None, :]]   # [p,4,4,4,O]


def _reduced_derivative(block, w, orders):
    """sum_{lmn} d^ox b_l(tx) d^oy b_m(ty) d^oz b_n(tz) beta_lmn for orders (ox, oy, oz)."""
    ox, oy, oz = orders
    return np.einsum("pl,pm,pn,plmno->po", w[0][ox], w[1][oy], w[2][oz], block)


def _weights(t, max_order):
    return [[weights(t[:, d], k) for k in range(max_order + 1)] for d in range(3)]


HESS_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def _orders(*axes):
    o = [0, 0, 0]
    for ax in axes:
        o[ax] += 1
    return tuple(o)


def eval_vgl(beta, lattice, pos, lap_beta=None, chunk=256):
    """V [P,O], grad [P,3,O], lap [P,O] of the spline with coefficients beta [N1][N2][N3][O].

    With ``lap_beta`` (a separate spline of the planewave Laplacian, Sec. III A),
    the Laplacian is that spline's value instead of the second derivatives.
    """
    beta = np.asarray(beta, dtype=np.float64)
    grid = beta.shape[:3]
    n_orb = beta.shape[3]
    jac, metric = jacobian(lattice, grid)
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    n_pts = i0.shape[0]
    v = np.empty((n_pts, n_orb))
    grad = np.empty((n_pts, 3, n_orb))
    lap = np.empty((n_pts, n_orb))
    for p0 in range(0, n_pts, chunk):
        sl = slice(p0, p0 + chunk)
        w = _weights(t[sl], 2)
        blk = _block(beta, i0[sl], grid)
        v[sl] = _reduced_derivative(blk, w, (0, 0, 0))
        g = np.stack([_reduced_derivative(blk, w, _orders(i)) for i in range(3)], axis=1)   # [p,3,O]
        grad[sl] = np.einsum("ia,pio->pao", jac, g)
        if lap_beta is None:
            acc = np.zeros((g.shape[0], n_orb))
            for i in range(3):
                for j in range(3):
                    acc += metric[i, j] * _reduced_derivative(blk, w, _orders(i, j))
            lap[sl] = acc
        else:
            lap[sl] = _reduced_derivative(_block(np.asarray(lap_beta, dtype=np.float64), i0[sl], grid),
                                          w, (0, 0, 0))
    v[~ok] = np.nan
    grad[~ok] = np.nan
    lap[~ok] = np.nan
    return v, grad, lap


def eval_v(beta, lattice, pos, chunk=256):
    """Values only, [P,O]."""
    beta = np.asarray(beta, dtype=np.float64)
    grid = beta.shape[:3]
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    v = np.empty((i0.shape[0], beta.shape[3]))
    for p0 in range(0, i0.shape[0], chunk):
        sl = slice(p0, p0 + chunk)
        w = _weights(t[sl], 0)
        v[sl] = _reduced_derivative(_block(beta, i0[sl], grid), w, (0, 0, 0))
    v[~ok] = np.nan
    return v


def eval_abs_bound(beta, lattice, pos, lap_beta=None, chunk=256):
    """Sum over the 64 terms of |weight| * |beta| for each output (V, grad, lap).

    Used to scale elementwise rounding-error tolerances: a sum of 64 products
    computed in precision u differs from the exact sum by at most about
    64 u times this quantity.
    """
    beta = np.abs(np.asarray(beta, dtype=np.float64))
    grid = beta.shape[:3]
    jac, metric = jacobian(lattice, grid)
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    n_pts, n_orb = i0.shape[0], beta.shape[3]
    v = np.empty((n_pts, n_orb))
    grad = np.empty((n_pts, 3, n_orb))
    lap = np.empty((n_pts, n_orb))
    for p0 in range(0, n_pts, chunk):
        sl = slice(p0, p0 + chunk)
        w = [[np.abs(x) for x in ax] for ax in _weights(t[sl], 2)]
        blk = _block(beta, i0[sl], grid)
        v[sl] = _reduced_derivative(blk, w, (0, 0, 0))
        g = np.stack([_reduced_derivative(blk, w, _orders(i)) for i in range(3)], axis=1)
        grad[sl] = np.einsum("ia,pio->pao", np.abs(jac), g)
        if lap_beta is None:
            acc = np.zeros((g.shape[0], n_orb))
            for i in range(3):
                for j in range(3):
                    acc += abs(metric[i, j]) * _reduced_derivative(blk, w, _orders(i, j))
            lap[sl] = acc
        else:
            lap[sl] = _reduced_derivative(_block(np.abs(np.asarray(lap_beta, dtype=np.float64)), i0[sl], grid),
                                          w, (0, 0, 0))
    return v, grad, lap


def coordinate_error_bound(beta, lattice, pos, du, lap_beta=None, chunk=256):
    """Bound on how much each output can move when the grid coordinates u_i of a point
    are perturbed by at most du [P,3] (rounding in the coordinate reduction).

    Uses the derivative one order higher, in absolute value:
      V:     sum_i du_i sum |d_i w||beta|
      grad:  sum_k |J_k alpha| sum_i du_i sum |d_i d_k w||beta|
      lap:   sum_jk |M_jk| sum_i du_i sum |d_i d_j d_k w||beta|
             (separate Laplacian spline: sum_i du_i sum |d_i w||beta_lap|)
    The third-derivative weights are piecewise constant, so the bound also covers
    points whose block index flips across a knot plane (the spline is C^2).
    """
    beta = np.abs(np.asarray(beta, dtype=np.float64))
    grid = beta.shape[:3]
    jac, metric = jacobian(lattice, grid)
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    du = np.asarray(du, dtype=np.float64)
    n_pts, n_orb = i0.shape[0], beta.shape[3]
    v = np.zeros((n_pts, n_orb))
    grad = np.zeros((n_pts, 3, n_orb))
    lap = np.zeros((n_pts, n_orb))
    for p0 in range(0, n_pts, chunk):
        sl = slice(p0, p0 + chunk)
        w = [[np.abs(x) for x in ax] for ax in _weights(t[sl], 3)]
        blk = _block(beta, i0[sl], grid)
        d = du[sl]
        for i in range(3):
            v[sl] += d[:, i, None] * _reduced_derivative(blk, w, _orders(i))
            for k in range(3):
                hik = _reduced_derivative(blk, w, _orders(i, k))
                grad[sl] += np.abs(jac[k])[None, :, None] * (d[:, i, None] * hik)[:, None, :]
                if lap_beta is None:
                    for j in range(3):
                        lap[sl] += abs(metric[j, k]) * d[:, i, None] * _reduced_derivative(blk, w, _orders(i, j, k))
            if lap_beta is not None:
                lblk = _block(np.abs(np.asarray(lap_beta, dtype=np.float64)), i0[sl], grid)
                lap[sl] += d[:, i, None] * _reduced_derivative(lblk, w, _orders(i))
    return v, grad, lap
