"""Piecewise-polynomial (pp) form of the periodic interpolating cubic spline (App. A,
Piecewise-polynomial-form splines).

Every grid point stores 2^3 = 8 numbers sigma^{kappa,mu,nu} (Eq. pp-splinecoefficients3): the grid
value (kappa, mu, nu) = (1,1,1); the second derivatives along one reduced axis, (2,1,1), (1,2,1) and
(1,1,2); the mixed fourth derivatives (2,2,1), (2,1,2), (1,2,2); and the sixth, (2,2,2).  Along one
axis the second derivatives solve the periodic system with rows (1, 4, 1) and corner elements against
6/h^2 times the second differences of the grid values, with h = 1 in grid units (App. A).  In three
dimensions a factor 2 in kappa, mu or nu applies that one-axis operator along x, y or z.

Evaluation (Eq. pp-splineinterpolation3) at reduced coordinate t in cell i0 uses the two grid points
i0 and i0 + 1 of every axis and the basis polynomials of Eq. pp-splinebasis,
    s^1_0 = 1 - t,   s^2_0 = -t^3/6 + t^2/2 - t/3,   s^1_1 = t,   s^2_1 = t^3/6 - t/6,
summing s^kappa_i(tx) s^mu_j(ty) s^nu_k(tz) sigma^{kappa,mu,nu} over the 8 corners and 8 kinds:
64 terms per orbital.  Derivatives follow by differentiating the polynomials and the chain rule of
Sec. II, as for the B-spline.

Stored order of the 8 numbers at a grid point: q = 4 (kappa - 1) + 2 (mu - 1) + (nu - 1).
"""
import numpy as np

from .evaluate import reduced_coordinates, jacobian

# Eq. pp-splinebasis: coefficients of t^3, t^2, t, 1, indexed [corner i][kappa - 1]
POLY = {(0, 1): [0.0, 0.0, -1.0, 1.0],
        (0, 2): [-1.0 / 6.0, 0.5, -1.0 / 3.0, 0.0],
        (1, 1): [0.0, 0.0, 1.0, 0.0],
        (1, 2): [1.0 / 6.0, 0.0, -1.0 / 6.0, 0.0]}


def basis(t, order=0):
    """d^order/dt^order s^kappa_i(t): array [..., 2 (corner i), 2 (kappa - 1)]."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty(t.shape + (2, 2))
    for i in (0, 1):
        for kappa in (1, 2):
            c = np.asarray(POLY[(i, kappa)])
            for _ in range(order):
                c = np.polyder(c)
            out[..., i, kappa - 1] = np.polyval(c, t)
    return out


def second_derivative_operator(n):
    """The one-axis map from grid values to the spline's second derivatives at the grid points:
    solve M sigma = 6 (f_{i-1} - 2 f_i + f_{i+1}), M periodic with rows (1, 4, 1)."""
    m = 4.0 * np.eye(n)
    d2 = -2.0 * np.eye(n)
    for i in range(n):
        m[i, (i - 1) % n] += 1.0
        m[i, (i + 1) % n] += 1.0
        d2[i, (i - 1) % n] += 1.0
        d2[i, (i + 1) % n] += 1.0
    return np.linalg.solve(m, 6.0 * d2)


def build_pp(f):
    """sigma [N1][N2][N3][8][O] from grid values f [N1][N2][N3][O] (real)."""
    f = np.asarray(f, dtype=np.float64)
    ops = [second_derivative_operator(n) for n in f.shape[:3]]
    out = np.empty(f.shape[:3] + (8,) + f.shape[3:])
    for kappa in (1, 2):
        for mu in (1, 2):
            for nu in (1, 2):
                v = f
                if kappa == 2:
                    v = np.einsum("ij,jklo->iklo", ops[0], v)
                if mu == 2:
                    v = np.einsum("ij,ajlo->ailo", ops[1], v)
                if nu == 2:
                    v = np.einsum("ij,abjo->abio", ops[2], v)
                out[..., 4 * (kappa - 1) + 2 * (mu - 1) + (nu - 1), :] = v
    return out


def _corners(sigma, i0, grid):
    ix = (i0[:, 0, None] + np.array([0, 1])) % grid[0]
    iy = (i0[:, 1, None] + np.array([0, 1])) % grid[1]
    iz = (i0[:, 2, None] + np.array([0, 1])) % grid[2]
    blk = sigma[ix[:, :, None, None], iy[:, None, :, None], iz[:, None, None, :]]     # [p,2,2,2,8,O]
    return blk.reshape(blk.shape[:4] + (2, 2, 2) + blk.shape[5:])                     # [p,i,j,k,ka,mu,nu,O]


def _reduced(blk, wx, wy, wz):
    return np.einsum("pia,pjb,pkc,pijkabco->po", wx, wy, wz, blk)


def eval_pp_vgl(sigma, lattice, pos, lap_sigma=None, chunk=256):
    """V [P,O], grad [P,3,O], lap [P,O] of the pp-spline sigma [N1][N2][N3][8][O].  With lap_sigma
    (the pp form of a separate Laplacian spline) the Laplacian is that spline's value."""
    sigma = np.asarray(sigma, dtype=np.float64)
    grid = sigma.shape[:3]
    n_orb = sigma.shape[4]
    jac, metric = jacobian(lattice, grid)
    i0, t, ok = reduced_coordinates(lattice, grid, pos)
    n_pts = i0.shape[0]
    v = np.empty((n_pts, n_orb))
    grad = np.empty((n_pts, 3, n_orb))
    lap = np.empty((n_pts, n_orb))
    for p0 in range(0, n_pts, chunk):
        sl = slice(p0, p0 + chunk)
        w = [[basis(t[sl, d], k) for k in range(3)] for d in range(3)]
        blk = _corners(sigma, i0[sl], grid)

        def red(ox, oy, oz):
            return _reduced(blk, w[0][ox], w[1][oy], w[2][oz])

        v[sl] = red(0, 0, 0)
        g = np.stack([red(1, 0, 0), red(0, 1, 0), red(0, 0, 1)], axis=1)
        grad[sl] = np.einsum("ia,pio->pao", jac, g)
        if lap_sigma is None:
            acc = np.zeros((g.shape[0], n_orb))
            for i in range(3):
                for j in range(3):
                    o = [0, 0, 0]
                    o[i] += 1
                    o[j] += 1
                    acc += metric[i, j] * red(*o)
            lap[sl] = acc
        else:
            lb = _corners(np.asarray(lap_sigma, dtype=np.float64), i0[sl], grid)
            lap[sl] = _reduced(lb, w[0][0], w[1][0], w[2][0])
    v[~ok] = np.nan
    grad[~ok] = np.nan
    lap[~ok] = np.nan
    return v, grad, lap


def eval_pp_v(sigma, lattice, pos):
    return eval_pp_vgl(sigma, lattice, pos)[0]
