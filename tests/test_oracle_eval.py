"""Pins of the oracle's evaluation: reduced coordinates, tensor product and chain rule."""
import numpy as np
import pytest

from oracle import build, evaluate, pw
from workloads import config, make_system

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])   # non-orthogonal cell, rows a_i


class CubicPoly:
    """q(r) = c0 + c.r + r^T Q r + sum T_abg r_a r_b r_g (total degree 3), analytic derivatives."""

    def __init__(self, rng):
        self.c0 = rng.standard_normal()
        self.c = rng.standard_normal(3)
        q = rng.standard_normal((3, 3)) * 0.1
        self.Q = q + q.T
        t = rng.standard_normal((3, 3, 3)) * 0.01
        self.T = sum(np.transpose(t, p) for p in
                     [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]) / 6

    def value(self, r):
        return (self.c0 + r @ self.c + np.einsum("pa,ab,pb->p", r, self.Q, r)
                + np.einsum("abg,pa,pb,pg->p", self.T, r, r, r))

    def grad(self, r):
        return self.c + 2 * r @ self.Q + 3 * np.einsum("abg,pb,pg->pa", self.T, r, r)

    def lap(self, r):
        return 2 * np.trace(self.Q) + 6 * np.einsum("aad,pd->p", self.T, r)


def test_cubic_reproduction_nonorthogonal():
    rng = np.random.default_rng(10)
    grid = (10, 11, 12)
    poly = CubicPoly(rng)
    # build on the extended grid, then trim one halo layer per axis in turn
    n = np.array(grid)
    ext = [np.arange(-1, k + 1) for k in grid]
    idx = np.stack(np.meshgrid(*ext, indexing="ij"), axis=-1)
    q = poly.value(((idx / n) @ SKEW).reshape(-1, 3)).reshape(idx.shape[:3])
    beta = q
    for ax in range(3):
        beta = np.moveaxis(beta, ax, 0)
        beta = beta[1:-1] - (beta[:-2] - 2 * beta[1:-1] + beta[2:]) / 6.0
        beta = np.moveaxis(beta, 0, ax)
    assert beta.shape == grid
    beta = beta[..., None]
    # points whose 4x4x4 block stays inside the filled (non-wrapping) index range
    u = rng.uniform(1.0, np.array(grid) - 3.0, size=(400, 3))
    pos = (u / n) @ SKEW
    v, g, lap = evaluate.eval_vgl(beta, SKEW, pos)
    scale = np.abs(poly.value(pos)).max()
    np.testing.assert_allclose(v[:, 0], poly.value(pos), atol=1e-12 * scale)
    np.testing.assert_allclose(g[:, :, 0], poly.grad(pos), atol=1e-11 * np.abs(poly.grad(pos)).max())
    np.testing.assert_allclose(lap[:, 0], poly.lap(pos), atol=1e-10 * np.abs(poly.lap(pos)).max())


def _random_spline(grid, n_orb, seed):
    rng = np.random.default_rng(seed)
    return build.build_interp(rng.standard_normal(tuple(grid) + (n_orb,)))


def _interior_points(lattice, grid, n, rng, lo=0.25, hi=0.75):
    cells = rng.integers(0, np.array(grid), size=(n, 3))
    u = cells + rng.uniform(lo, hi, size=(n, 3))
    return (u / np.array(grid)) @ lattice


def test_gradient_laplacian_finite_differences():
    grid = (8, 9, 10)
    beta = _random_spline(grid, 3, 11)
    rng = np.random.default_rng(12)
    pos = _interior_points(SKEW, grid, 50, rng)
    v, g, lap = evaluate.eval_vgl(beta, SKEW, pos)
    d = 1e-4
    gfd = np.empty_like(g)
    lfd = np.zeros_like(lap)
    for a in range(3):
        e = np.zeros(3)
        e[a] = d
        vp = evaluate.eval_v(beta, SKEW, pos + e)
        vm = evaluate.eval_v(beta, SKEW, pos - e)
        gfd[:, a] = (vp - vm) / (2 * d)
        lfd += (vp - 2 * v + vm) / d**2
    np.testing.assert_allclose(g, gfd, atol=1e-7 * np.abs(g).max())
    np.testing.assert_allclose(lap, lfd, atol=1e-5 * np.abs(lap).max())


def test_periodicity_and_folding():
    grid = (8, 9, 10)
    beta = _random_spline(grid, 2, 13)
    rng = np.random.default_rng(14)
    pos = rng.uniform(-20, 20, size=(100, 3))
    shifts = rng.integers(-3, 4, size=(100, 3)) @ SKEW
    a = evaluate.eval_vgl(beta, SKEW, pos)
    b = evaluate.eval_vgl(beta, SKEW, pos + shifts)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, atol=1e-11 * np.abs(x).max())


def test_reduced_coordinate_edges():
    grid = (8, 8, 8)
    lat = np.eye(3) * 4.0
    pos = np.array([[-1e-300, 0.0, 0.0],       # s rounds to 1.0 after folding: wraps to index 0
                    [4.0, 8.0, -4.0],          # whole lattice vectors
                    [0.5, 1.0, 3.5],           # exactly on grid planes
                    [np.nan, 0.0, 0.0],
                    [0.0, np.inf, 0.0]])
    i0, t, ok = evaluate.reduced_coordinates(lat, grid, pos)
    assert ok.tolist() == [True, True, True, False, False]
    assert i0[0].tolist() == [0, 0, 0] and t[0].tolist() == [0.0, 0.0, 0.0]
    assert i0[1].tolist() == [0, 0, 0]
    assert i0[2].tolist() == [1, 2, 7] and t[2].tolist() == [0.0, 0.0, 0.0]
    assert np.all((i0 >= 0) & (i0 < 8)) and np.all((t >= 0) & (t < 1))
    beta = _random_spline(grid, 2, 15)
    v, g, lap = evaluate.eval_vgl(beta, lat, pos)
    assert np.isnan(v[3:]).all() and np.isnan(g[3:]).all() and np.isnan(lap[3:]).all()
    assert np.isfinite(v[:3]).all()


def test_derivatives_at_knots_single_planewave():
    # f = exp(i theta.j): at a knot, d/du = i sin(theta)/lambda * f and d2/du2 = (2 cos theta - 2)/lambda * f
    grid = (8, 10, 12)
    lengths = np.array([5.0, 6.0, 7.5])
    lat = np.diag(lengths)
    n = np.array(grid)
    theta = 2 * np.pi * np.array([1, -2, 3]) / n
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in grid], indexing="ij"), axis=-1)
    phase = idx @ theta
    f = np.stack([np.cos(phase), np.sin(phase)], axis=-1)
    beta = build.build_interp(f)
    lam = (4 + 2 * np.cos(theta)) / 6
    rng = np.random.default_rng(16)
    k = rng.integers(0, n, size=(60, 3))
    pos = (k / n) * lengths
    v, g, lap = evaluate.eval_vgl(beta, lat, pos)
    z = np.exp(1j * (k @ theta))
    scale = n / lengths                         # d u / d r per axis
    for a in range(3):
        dz = 1j * np.sin(theta[a]) / lam[a] * z * scale[a]
        np.testing.assert_allclose(g[:, a, 0], dz.real, atol=1e-13)
        np.testing.assert_allclose(g[:, a, 1], dz.imag, atol=1e-13)
    lz = sum((2 * np.cos(theta[a]) - 2) / lam[a] * scale[a] ** 2 for a in range(3)) * z
    np.testing.assert_allclose(lap[:, 0], lz.real, atol=1e-12)
    np.testing.assert_allclose(lap[:, 1], lz.imag, atol=1e-12)


def test_separate_laplacian_single_planewave_everywhere():
    grid = (8, 8, 8)
    lat = SKEW
    n = np.array(grid)
    miller = np.array([1, 1, -2])
    gvec = 2 * np.pi * np.linalg.inv(lat) @ miller
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in grid], indexing="ij"), axis=-1)
    phase = idx @ (2 * np.pi * miller / n)
    f = np.cos(phase)[..., None]
    beta = build.build_interp(f)
    lap_beta = build.build_interp(-(gvec @ gvec) * f)
    pos = np.random.default_rng(17).uniform(-10, 10, size=(200, 3))
    v, _, lap = evaluate.eval_vgl(beta, lat, pos, lap_beta=lap_beta)
    np.testing.assert_allclose(lap, -(gvec @ gvec) * v, atol=1e-13 * (gvec @ gvec))


def test_pw_laplacian_and_gradient():
    s = config(0).system
    pos = s.positions(30)
    v, g, lap = pw.pw_vgl(s.gvecs, s.coef, pos)
    # one planewave term at a time: lap = -|G|^2 value
    for j in (0, 7, 100):
        cj = np.zeros_like(s.coef)
        cj[:, j] = s.coef[:, j]
        vj, _, lj = pw.pw_vgl(s.gvecs, cj, pos)
        np.testing.assert_allclose(lj, -(s.gvecs[j] @ s.gvecs[j]) * vj, atol=1e-14)
    d = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = d
        fd = (pw.pw_value(s.gvecs, s.coef, pos + e) - pw.pw_value(s.gvecs, s.coef, pos - e)) / (2 * d)
        np.testing.assert_allclose(g[:, a], fd, atol=1e-8 * np.abs(g).max())
    # orbitals are real: the imaginary part of the raw sum vanishes
    e = np.exp(1j * pos @ s.gvecs.T)
    assert np.abs((e @ s.coef.T).imag).max() < 1e-12 * np.abs(v).max()


def test_convergence_order_with_grid_spacing():
    base = config(0).system
    errs = []
    pos = base.positions(300)
    vp, gp, lp = pw.pw_vgl(base.gvecs, base.coef, pos)
    for n in (24, 48):
        s = make_system("conv", base.lattice, (n, n, n), base.n_orb, base.gcut, base.decay, base.seed_key)
        beta = build.build_interp(s.grid_values())
        v, g, lap = evaluate.eval_vgl(beta, s.lattice, pos)
        errs.append([np.abs(v - vp).max(), np.abs(g - gp).max(), np.abs(lap - lp).max()])
    ratio = np.array(errs[0]) / np.array(errs[1])
    assert ratio[0] > 10 and ratio[1] > 5 and ratio[2] > 2.5, ratio


def test_spline_close_to_planewave_config0():
    w = config(0)
    s = w.system
    beta = build.build_interp(s.grid_values())
    pos = w.positions()[:500]
    v, g, lap = evaluate.eval_vgl(beta, s.lattice, pos)
    vp, gp, lp = pw.pw_vgl(s.gvecs, s.coef, pos)
    rel = [np.abs(a - b).max() / np.abs(b).max() for a, b in ((v, vp), (g, gp), (lap, lp))]
    assert rel[0] < 1e-2 and rel[1] < 5e-2 and rel[2] < 0.2, rel


def test_coordinate_error_bound_covers_small_shifts():
    grid = (8, 9, 10)
    beta = _random_spline(grid, 3, 18)
    rng = np.random.default_rng(19)
    pos = rng.uniform(-15, 15, size=(200, 3))
    n = np.array(grid)
    du = np.full((200, 3), 1e-6)
    # move every point by up to du in grid units (here along the cell axes)
    shift = (rng.uniform(-1, 1, size=(200, 3)) * du / n) @ SKEW
    a = evaluate.eval_vgl(beta, SKEW, pos)
    b = evaluate.eval_vgl(beta, SKEW, pos + shift)
    bounds = evaluate.coordinate_error_bound(beta, SKEW, pos, du)
    for x, y, bd in zip(a, b, bounds):
        assert np.all(np.abs(x - y) <= 1.01 * bd + 1e-15)
