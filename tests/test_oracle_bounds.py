"""Pins of the oracle's rounding-error scales (evaluate.eval_abs_bound, lagrange.eval_abs_bound).

These functions set the width of every elementwise kernel-parity tolerance: for each output q
they return sum_{lmn} |w^q_lmn| |beta_lmn| (with |J| and |M| in the chain rule), the scale of
the rounding error of a 64-term sum (App. A, Eq. b-splineapproximation, Eq. lagrangeinterpolation3).
An overestimate would silently loosen parity, an underestimate would make it flaky; both are
checked here against what the mathematics fixes:
  - the bound dominates |output| for any table (triangle inequality);
  - it is attained (tight) where the chain rule does not mix axes: for a table whose signs
    match the weights' signs at a point, the output equals the bound there;
  - it equals a brute-force sum over the 64 block points, written with scalar loops from the
    grid-centred basis functions b, b', b'' (not from the oracle's vectorized weights);
  - the Lagrange coordinate term equals |d value / d u| times du for a sign-matched table,
    measured by central differences of the oracle's own value function inside one cell.
"""
import numpy as np

from oracle import bspline, evaluate, lagrange

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])   # rows a_i
ORTHO = np.diag([6.5, 7.25, 8.0])
GRID = (7, 8, 9)


def _points(lattice, n, seed):
    rng = np.random.default_rng(seed)
    s = rng.uniform(-1.5, 2.5, size=(n, 3))          # crystal coordinates, several images
    return s @ lattice


def _reduced(lattice, grid, pos):
    i0, t, ok = evaluate.reduced_coordinates(lattice, grid, pos)
    assert ok.all()
    return i0, t


def test_value_bound_equals_value_of_nonnegative_table():
    """B-spline weights are non-negative, so for beta >= 0 the V bound is V itself."""
    rng = np.random.default_rng(1)
    beta = np.abs(rng.standard_normal(GRID + (3,)))
    pos = _points(SKEW, 300, 2)
    v, _, _ = evaluate.eval_vgl(beta, SKEW, pos)
    bv, _, _ = evaluate.eval_abs_bound(beta, SKEW, pos)
    np.testing.assert_allclose(bv, v, rtol=1e-14, atol=0)
    # and for a signed table the bound is V of |beta|
    signed = beta * rng.choice([-1.0, 1.0], size=beta.shape)
    bv2, _, _ = evaluate.eval_abs_bound(signed, SKEW, pos)
    np.testing.assert_allclose(bv2, v, rtol=1e-14, atol=0)


def test_bounds_dominate_outputs():
    rng = np.random.default_rng(3)
    beta = rng.standard_normal(GRID + (4,))
    lbeta = rng.standard_normal(GRID + (4,))
    pos = _points(SKEW, 400, 4)
    for lb in (None, lbeta):
        out = evaluate.eval_vgl(beta, SKEW, pos, lap_beta=lb)
        bnd = evaluate.eval_abs_bound(beta, SKEW, pos, lap_beta=lb)
        for o, b in zip(out, bnd):
            assert np.all(np.abs(o) <= b * (1 + 1e-13) + 1e-300)
            # and not absurdly loose: on random signs the bound is within ~100x of |output|
            assert np.median(b / np.maximum(np.abs(o), 1e-300)) < 100


def _brute_force(beta, lattice, pos):
    """sum over l, m, n in {-1..2} of |weight| |beta| for V, each gradient component and the
    Laplacian, with scalar loops and the grid-centred basis b(t - l) and its derivatives."""
    grid = beta.shape[:3]
    a = np.asarray(lattice, dtype=np.float64).T
    jac = np.asarray(grid, dtype=np.float64)[:, None] * np.linalg.inv(a)
    metric = jac @ jac.T
    fns = (bspline.b, bspline.db, bspline.d2b)
    i0, t = _reduced(lattice, grid, pos)
    n_pts, n_orb = pos.shape[0], beta.shape[3]
    v = np.zeros((n_pts, n_orb))
    grad = np.zeros((n_pts, 3, n_orb))
    lap = np.zeros((n_pts, n_orb))
    for p in range(n_pts):
        for l in (-1, 0, 1, 2):
            for m in (-1, 0, 1, 2):
                for n in (-1, 0, 1, 2):
                    row = np.abs(beta[(i0[p, 0] + l) % grid[0], (i0[p, 1] + m) % grid[1], (i0[p, 2] + n) % grid[2]])
                    offs = (l, m, n)

                    def w(orders):
                        x = 1.0
                        for ax in range(3):
                            x *= float(fns[orders[ax]](t[p, ax] - offs[ax]))
                        return abs(x)

                    v[p] += w((0, 0, 0)) * row
                    for i in range(3):
                        e = [0, 0, 0]
                        e[i] = 1
                        for al in range(3):
                            grad[p, al] += abs(jac[i, al]) * w(tuple(e)) * row
                        for j in range(3):
                            f = [0, 0, 0]
                            f[i] += 1
                            f[j] += 1
                            lap[p] += abs(metric[i, j]) * w(tuple(f)) * row
    return v, grad, lap


def test_bounds_equal_brute_force_sum():
    rng = np.random.default_rng(5)
    beta = rng.standard_normal(GRID + (2,))
    pos = _points(SKEW, 12, 6)
    got = evaluate.eval_abs_bound(beta, SKEW, pos)
    ref = _brute_force(beta, SKEW, pos)
    for name, g, r in zip(("V", "grad", "lap"), got, ref):
        np.testing.assert_allclose(g, r, rtol=1e-13, atol=0, err_msg=name)


def _sign_matched_table(grid, n_orb, i0, t, orders, rng):
    """Table whose orbital o has, on the block of point o, the signs of the weights of the
    derivative `orders` at that point (other entries random).  Point o's output for orbital o is
    then sum |w||beta| exactly."""
    beta = rng.standard_normal(grid + (n_orb,))
    fns = (bspline.b, bspline.db, bspline.d2b)
    for o in range(n_orb):
        for l in (-1, 0, 1, 2):
            for m in (-1, 0, 1, 2):
                for n in (-1, 0, 1, 2):
                    x = 1.0
                    for ax, off in enumerate((l, m, n)):
                        x *= float(fns[orders[ax]](t[o, ax] - off))
                    idx = ((i0[o, 0] + l) % grid[0], (i0[o, 1] + m) % grid[1], (i0[o, 2] + n) % grid[2], o)
                    beta[idx] = np.sign(x) * abs(beta[idx])
    return beta


def test_gradient_bound_attained_on_orthogonal_cell():
    """J is diagonal in an orthogonal cell, so grad_alpha = J_aa d_a phi and the bound
    |J_aa| sum |d_a w||beta| is reached by the sign-matched table."""
    rng = np.random.default_rng(7)
    n_pts = 6
    pos = _points(ORTHO, n_pts, 8)
    i0, t = _reduced(ORTHO, GRID, pos)
    for axis in range(3):
        orders = [0, 0, 0]
        orders[axis] = 1
        beta = _sign_matched_table(GRID, n_pts, i0, t, tuple(orders), rng)
        _, g, _ = evaluate.eval_vgl(beta, ORTHO, pos)
        _, bg, _ = evaluate.eval_abs_bound(beta, ORTHO, pos)
        diag = np.arange(n_pts)
        got = np.abs(g[diag, axis, diag])
        np.testing.assert_allclose(got, bg[diag, axis, diag], rtol=1e-13)
        # the two other components are strictly below their bounds (signs do not match them)
        for other in set(range(3)) - {axis}:
            assert np.all(np.abs(g[diag, other, diag]) < bg[diag, other, diag])


def test_laplacian_bound_attained_on_one_axis_table():
    """In an orthogonal cell lap = sum_i M_ii d_i^2 phi.  A table that varies along x only
    (beta_lmn = beta_l) has d_y^2 phi = d_z^2 phi = 0, and its x part reaches
    M_xx sum |d_x^2 w| |beta|.  The bound's y and z parts are sum over |d^2 w| of those axes times
    |beta|, which for a constant-along-the-axis table are M_yy * sum_m |b''_m| * (sum |b_l''|...).
    So check lap = M_xx S_x exactly and that the bound is S_x M_xx plus the two known surplus terms."""
    rng = np.random.default_rng(9)
    n_pts = 5
    pos = _points(ORTHO, n_pts, 10)
    i0, t = _reduced(ORTHO, GRID, pos)
    jac = np.asarray(GRID, dtype=np.float64)[:, None] * np.linalg.inv(ORTHO.T)
    metric = jac @ jac.T
    for p in range(n_pts):
        prof = np.abs(rng.standard_normal(GRID[0])) + 0.1
        d2x = bspline.weights(t[p, 0], 2)
        rows = (i0[p, 0] + bspline.OFFSETS) % GRID[0]
        prof[rows] = np.sign(d2x) * prof[rows]
        beta = np.broadcast_to(prof[:, None, None, None], GRID + (1,)).copy()
        _, _, lap = evaluate.eval_vgl(beta, ORTHO, pos[p:p + 1])
        _, _, bl = evaluate.eval_abs_bound(beta, ORTHO, pos[p:p + 1])
        sx = float(np.sum(np.abs(d2x) * np.abs(prof[rows])))
        np.testing.assert_allclose(lap[0, 0], metric[0, 0] * sx, rtol=1e-13)
        # surplus from the y and z axes: M_ii sum_l |b_l(tx)| |beta_l| * sum_m |b''_m(t_i)|
        vx = float(np.sum(bspline.weights(t[p, 0]) * np.abs(prof[rows])))
        surplus = sum(metric[i, i] * vx * float(np.sum(np.abs(bspline.weights(t[p, i], 2)))) for i in (1, 2))
        np.testing.assert_allclose(bl[0, 0], metric[0, 0] * sx + surplus, rtol=1e-13)


def test_separate_laplacian_bound_is_value_bound_of_laplacian_table():
    rng = np.random.default_rng(11)
    beta = rng.standard_normal(GRID + (2,))
    lbeta = np.abs(rng.standard_normal(GRID + (2,)))
    pos = _points(SKEW, 50, 12)
    _, _, bl = evaluate.eval_abs_bound(beta, SKEW, pos, lap_beta=lbeta)
    vl, _, _ = evaluate.eval_vgl(lbeta, SKEW, pos)
    np.testing.assert_allclose(bl, vl, rtol=1e-14)


# ----------------------------------------------------------------------------- Lagrange


def test_lagrange_bound_dominates_and_is_attained():
    rng = np.random.default_rng(13)
    n_pts = 8
    pos = _points(SKEW, n_pts, 14)
    i0, t = _reduced(SKEW, GRID, pos)
    vals = rng.standard_normal(GRID + (n_pts,))
    acc, _ = lagrange.eval_abs_bound(vals, SKEW, pos)
    out = lagrange.eval_values(vals, SKEW, pos)
    assert np.all(np.abs(out) <= acc * (1 + 1e-13))
    # sign-matched values: orbital o at point o reaches the bound
    for o in range(n_pts):
        wx = lagrange.weights(t[o, 0])
        wy = lagrange.weights(t[o, 1])
        wz = lagrange.weights(t[o, 2])
        for a, l in enumerate(bspline.OFFSETS):
            for b, m in enumerate(bspline.OFFSETS):
                for c, n in enumerate(bspline.OFFSETS):
                    idx = ((i0[o, 0] + l) % GRID[0], (i0[o, 1] + m) % GRID[1], (i0[o, 2] + n) % GRID[2], o)
                    vals[idx] = np.sign(wx[a] * wy[b] * wz[c]) * abs(vals[idx])
    acc, _ = lagrange.eval_abs_bound(vals, SKEW, pos)
    out = lagrange.eval_values(vals, SKEW, pos)
    diag = np.arange(n_pts)
    np.testing.assert_allclose(out[diag, diag], acc[diag, diag], rtol=1e-13)


def test_lagrange_coordinate_term_is_derivative_magnitude():
    """With du = e_axis and values whose signs match d_axis(ell ell ell) at the point, the
    coordinate term equals |d value / d u_axis|, measured by a central difference of the
    oracle's value function inside the point's cell."""
    rng = np.random.default_rng(15)
    n_pts = 6
    pos = _points(ORTHO, n_pts, 16)
    i0, t = _reduced(ORTHO, GRID, pos)
    t = np.clip(t, 0.05, 0.95)                       # keep the stencil inside one cell
    n = np.asarray(GRID, dtype=np.float64)
    pos = ((i0 + t) / n) @ ORTHO
    for axis in range(3):
        vals = rng.standard_normal(GRID + (n_pts,))
        for o in range(n_pts):
            w = [lagrange.weights(t[o, ax], 1 if ax == axis else 0) for ax in range(3)]
            for a, l in enumerate(bspline.OFFSETS):
                for b, m in enumerate(bspline.OFFSETS):
                    for c, k in enumerate(bspline.OFFSETS):
                        idx = ((i0[o, 0] + l) % GRID[0], (i0[o, 1] + m) % GRID[1], (i0[o, 2] + k) % GRID[2], o)
                        vals[idx] = np.sign(w[0][a] * w[1][b] * w[2][c]) * abs(vals[idx])
        du = np.zeros((n_pts, 3))
        du[:, axis] = 1.0
        _, coord = lagrange.eval_abs_bound(vals, ORTHO, pos, du)
        h = 1e-5
        step = np.zeros(3)
        step[axis] = h / n[axis]
        fd = (lagrange.eval_values(vals, ORTHO, pos + step @ ORTHO)
              - lagrange.eval_values(vals, ORTHO, pos - step @ ORTHO)) / (2 * h)
        diag = np.arange(n_pts)
        np.testing.assert_allclose(np.abs(fd[diag, diag]), coord[diag, diag], rtol=1e-7)
