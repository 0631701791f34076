"""Pins of the oracle's other representations: cubic Lagrange interpolation (App. A), separate
gradient and Laplacian interpolants (Sec. III A, Fig. 1), and Bloch orbitals e^{ik.r} u(r)
(Sec. I), against the paper's printed polynomials, closed forms, the Bloch theorem, finite
differences and the planewave sums."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import lagrange, separate, bloch, build, evaluate, pw, smoothing
from workloads import config, make_system
from workloads.configs import fcc_primitive, A_SI

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])


def _golden_lagrange():
    rows, pieces = {}, {}
    with open(os.path.join(GOLDEN, "lagrange_basis_paper.txt")) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "offset":
                rows[int(f[1])] = [float(Fraction(x)) for x in f[2:]]
            else:
                pieces[f[0]] = [float(Fraction(x)) for x in f[1:]]
    return rows, pieces


# ---------------------------------------------------------------- Lagrange basis
def test_lagrange_weights_match_printed_polynomials():
    rows, pieces = _golden_lagrange()
    t = np.linspace(0.0, 0.999, 101)
    w = lagrange.weights(t)
    for a, l in enumerate((-1, 0, 1, 2)):
        np.testing.assert_allclose(w[:, a], np.polyval(rows[l], t), atol=1e-15)
    # grid-centred form: ell_l(t) = ell(t - l)
    def centred(xi):
        x = np.abs(xi)
        inner = np.polyval([pieces["inner"][0], pieces["inner"][1], pieces["inner"][2], pieces["inner"][3]], x)
        outer = np.polyval([pieces["outer"][0], pieces["outer"][1], pieces["outer"][2], pieces["outer"][3]], x)
        return np.where(x < 1, inner, np.where(x < 2, outer, 0.0))
    for a, l in enumerate((-1, 0, 1, 2)):
        np.testing.assert_allclose(w[:, a], centred(t - l), atol=1e-15)


def test_lagrange_derivative_weights_match_printed_polynomials():
    rows, _ = _golden_lagrange()
    t = np.linspace(0.0, 0.999, 101)
    dw = lagrange.weights(t, 1)
    for a, l in enumerate((-1, 0, 1, 2)):
        np.testing.assert_allclose(dw[:, a], np.polyval(np.polyder(rows[l]), t), atol=1e-14)
    np.testing.assert_allclose(dw.sum(1), 0.0, atol=1e-14)


def test_lagrange_interpolates_and_reproduces_cubics():
    np.testing.assert_array_equal(lagrange.weights(np.array([0.0]))[0], [0.0, 1.0, 0.0, 0.0])
    rng = np.random.default_rng(60)
    t = rng.random(200)
    w = lagrange.weights(t)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-15)
    for _ in range(5):
        c = rng.standard_normal(4)
        np.testing.assert_allclose(w @ np.polyval(c, np.array([-1.0, 0, 1, 2])), np.polyval(c, t), atol=1e-13)


def test_lagrange_tricubic_reproduction_in_skewed_cell():
    grid = (9, 8, 10)
    rng = np.random.default_rng(61)
    c = rng.standard_normal((4, 4, 4))              # q(x,y,z) = sum c_abc x^a y^b z^c in grid units
    ii = np.stack(np.meshgrid(*[np.arange(n, dtype=float) for n in grid], indexing="ij"), -1)
    def q(u):
        return sum(c[a, b, cc] * u[..., 0] ** a * u[..., 1] ** b * u[..., 2] ** cc
                   for a in range(4) for b in range(4) for cc in range(4))
    vals = q(ii)[..., None]
    # points whose block i0-1 .. i0+2 stays inside the grid (no periodic wrap)
    u = rng.uniform(1.0, np.array(grid) - 3.0, size=(300, 3))
    pos = (u / np.array(grid)) @ SKEW
    got = lagrange.eval_values(vals, SKEW, pos)[:, 0]
    np.testing.assert_allclose(got, q(u), rtol=1e-11, atol=1e-11 * np.abs(q(u)).max())


def test_lagrange_grid_points_and_periodicity():
    s = config(0).system
    f = s.grid_values()
    idx = np.random.default_rng(62).integers(0, 16, size=(40, 3))
    r = (idx / 16.0) @ s.lattice
    np.testing.assert_allclose(lagrange.eval_values(f, s.lattice, r), f[idx[:, 0], idx[:, 1], idx[:, 2]],
                               atol=1e-13 * np.abs(f).max())
    pos = s.positions(100)
    base = lagrange.eval_values(f, s.lattice, pos)
    for i in range(3):
        np.testing.assert_allclose(lagrange.eval_values(f, s.lattice, pos + s.lattice[i]), base,
                                   atol=1e-12 * np.abs(base).max())


def test_lagrange_converges_fourth_order():
    lat = np.diag([6.0, 6.0, 6.0])
    errs = []
    for n in (16, 32):
        s = make_system("conv", lat, (n, n, n), 2, 2.5, 2.0, (8, 8))
        pos = s.positions(300)
        v = pw.pw_value(s.gvecs, s.coef, pos)
        errs.append(np.abs(lagrange.eval_values(s.grid_values(), lat, pos) - v).max())
    assert errs[0] / errs[1] > 10.0, errs          # h^4: 16x asymptotically


# ---------------------------------------------------------------- separate interpolants
def _sep_tables(s, basis):
    vals = [s.grid_values()] + list(s.grid_gradient()) + [s.grid_laplacian()]
    if basis == "bspline":
        return [build.build_interp(np.ascontiguousarray(v)) for v in vals]
    return vals


@pytest.mark.parametrize("basis", ["bspline", "lagrange"])
def test_separate_interpolants_exact_at_grid_points(basis):
    s = make_system("sep", SKEW, (10, 9, 11), 3, 2.2, 2.0, (9, 9))
    assert s.nyquist_ok()
    tabs = _sep_tables(s, basis)
    idx = np.random.default_rng(63).integers(0, np.array(s.grid), size=(30, 3))
    r = (idx / np.array(s.grid)) @ SKEW
    v, g, l = separate.eval_separate(tabs, SKEW, r, basis)
    pv, pg, pl = pw.pw_vgl(s.gvecs, s.coef, r)
    for got, ref in ((v, pv), (g, pg), (l, pl)):
        np.testing.assert_allclose(got, ref, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("basis", ["bspline", "lagrange"])
def test_separate_interpolants_approach_planewave(basis):
    s = config(0).system
    pos = s.positions(200)
    v, g, l = separate.eval_separate(_sep_tables(s, basis), s.lattice, pos, basis)
    pv, pg, pl = pw.pw_vgl(s.gvecs, s.coef, pos)
    for got, ref, tol in ((v, pv, 0.05), (g, pg, 0.05), (l, pl, 0.1)):
        assert np.abs(got - ref).mean() / np.abs(ref).mean() < tol


def test_separate_laplacian_beats_derivative_laplacian():
    s = config(0).system
    pos = s.positions(300)
    _, _, pl = pw.pw_vgl(s.gvecs, s.coef, pos)
    _, _, l_sep = separate.eval_separate(_sep_tables(s, "bspline"), s.lattice, pos, "bspline")
    _, _, l_der = evaluate.eval_vgl(build.build_interp(s.grid_values()), s.lattice, pos)
    assert np.abs(l_sep - pl).mean() < np.abs(l_der - pl).mean()


# ---------------------------------------------------------------- Bloch orbitals
def test_planewave_bloch_sums():
    s = config(6).system
    pos = s.positions(20)
    v, g, l = bloch.pw_bloch_vgl(s.gvecs, s.coef, s.k, pos)
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (bloch.pw_bloch_vgl(s.gvecs, s.coef, s.k, pos + e)[0] - bloch.pw_bloch_vgl(s.gvecs, s.coef, s.k, pos - e)[0]) / (2 * h)
        np.testing.assert_allclose(g[:, a], fd, atol=1e-7 * np.abs(g).max())
    # one planewave: lap = -|k+G|^2 phi
    one = np.zeros_like(s.coef[:1])
    one[0, 7] = 1.0
    v1, _, l1 = bloch.pw_bloch_vgl(s.gvecs, one, s.k, pos)
    q = s.gvecs[7] + s.k
    np.testing.assert_allclose(l1, -(q @ q) * v1, rtol=1e-13)
    # Bloch theorem
    for i in range(3):
        vs = bloch.pw_bloch_vgl(s.gvecs, s.coef, s.k, pos + s.lattice[i])[0]
        np.testing.assert_allclose(vs, np.exp(1j * s.k @ s.lattice[i]) * v, atol=1e-12 * np.abs(v).max())


def _bloch_case(key=6, lap=False):
    s = config(key).system
    beta = build.build_interp(np.ascontiguousarray(s.grid_values().real)) + \
        1j * build.build_interp(np.ascontiguousarray(s.grid_values().imag))
    lb = None
    if lap:
        w = s.grid_laplacian()
        lb = build.build_interp(np.ascontiguousarray(w.real)) + 1j * build.build_interp(np.ascontiguousarray(w.imag))
    return s, beta, lb


@pytest.mark.parametrize("lap", [False, True])
def test_bloch_spline_obeys_bloch_theorem(lap):
    s, beta, lb = _bloch_case(lap=lap)
    pos = s.positions(80)
    base = bloch.eval_bloch_vgl(beta, s.lattice, s.k, pos, lap_beta=lb)
    for i in range(3):
        shifted = bloch.eval_bloch_vgl(beta, s.lattice, s.k, pos + s.lattice[i], lap_beta=lb)
        ph = np.exp(1j * s.k @ s.lattice[i])
        for a, b in zip(shifted, base):
            np.testing.assert_allclose(a, ph * b, atol=1e-11 * np.abs(b).max())
    assert np.abs(s.k @ s.lattice[0] % (2 * np.pi)) > 0.1      # a genuine twist, not a Gamma point


def test_bloch_spline_product_rule_by_finite_differences():
    s, beta, _ = _bloch_case()
    rng = np.random.default_rng(64)
    cells = rng.integers(0, 16, size=(40, 3))
    pos = ((cells + rng.uniform(0.25, 0.75, size=(40, 3))) / 16.0) @ s.lattice     # off the knot planes
    v, g, l = bloch.eval_bloch_vgl(beta, s.lattice, s.k, pos)
    h = 1e-4
    lap_fd = np.zeros_like(v)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        vp = bloch.eval_bloch_v(beta, s.lattice, s.k, pos + e)
        vm = bloch.eval_bloch_v(beta, s.lattice, s.k, pos - e)
        np.testing.assert_allclose(g[:, a], (vp - vm) / (2 * h), atol=1e-6 * np.abs(g).max())
        lap_fd += (vp - 2 * v + vm) / h**2
    np.testing.assert_allclose(l, lap_fd, atol=1e-4 * np.abs(l).max())
    np.testing.assert_allclose(bloch.eval_bloch_v(beta, s.lattice, s.k, pos), v, rtol=0, atol=1e-14 * np.abs(v).max())


def test_bloch_separate_laplacian_of_one_planewave():
    # u = e^{iG.r}: w = -|k+G|^2 u exactly, and the build is linear, so the separate Laplacian
    # equals -|k+G|^2 times the value everywhere
    s = config(6).system
    one = np.zeros_like(s.coef[:1])
    one[0, 11] = 1.0
    from workloads.synth import _grid_from_coef
    u = _grid_from_coef(s.miller, one, s.grid, keep_complex=True)
    q = s.gvecs[11] + s.k
    bu = build.build_interp(np.ascontiguousarray(u.real)) + 1j * build.build_interp(np.ascontiguousarray(u.imag))
    pos = s.positions(50)
    v, _, l = bloch.eval_bloch_vgl(bu, s.lattice, s.k, pos, lap_beta=-(q @ q) * bu)
    np.testing.assert_allclose(l, -(q @ q) * v, atol=1e-13 * np.abs(l).max())


@pytest.mark.parametrize("kind", ["derivative", "separate_lap", "separate_all"])
def test_bloch_spline_approaches_planewave(kind):
    s, beta, lb = _bloch_case(lap=(kind == "separate_lap"))
    pos = s.positions(200)
    if kind == "separate_all":
        tabs = [s.grid_values()] + list(s.grid_gradient()) + [s.grid_laplacian()]
        tabs = [build.build_interp(np.ascontiguousarray(t.real)) + 1j * build.build_interp(np.ascontiguousarray(t.imag))
                for t in tabs]
        got = bloch.eval_bloch_separate(tabs, s.lattice, s.k, pos)
    else:
        got = bloch.eval_bloch_vgl(beta, s.lattice, s.k, pos, lap_beta=lb)
    ref = bloch.pw_bloch_vgl(s.gvecs, s.coef, s.k, pos)
    tols = (0.02, 0.05, 0.3 if kind == "derivative" else 0.05)
    for a, b, tol in zip(got, ref, tols):
        assert np.abs(a - b).mean() / np.abs(b).mean() < tol, (kind, np.abs(a - b).mean() / np.abs(b).mean())


def test_bloch_smoothing_fourier_components():
    # complex smoothing coefficients: the fundamental Fourier components of u equal c_G
    lat = fcc_primitive(A_SI)
    s = make_system("bl-smooth", lat, (10, 10, 10), 1, 1.6, 2.0, (7, 8), kvec=(np.pi / A_SI) * np.array([1.0, 0, 0]))
    assert s.nyquist_ok()
    beta = smoothing.build_smoothing(s.miller, s.coef, s.grid, keep_complex=True)
    xg, wg = np.polynomial.legendre.leggauss(10)
    xg, wg = (xg + 1) / 2, wg / 2
    n = np.array(s.grid)
    cells = np.stack(np.meshgrid(*[np.arange(k) for k in s.grid], indexing="ij"), -1).reshape(-1, 3)
    nodes = np.stack(np.meshgrid(xg, xg, xg, indexing="ij"), -1).reshape(-1, 3)
    wts = np.einsum("i,j,k->ijk", wg, wg, wg).reshape(-1)
    u = (cells[:, None, :] + nodes[None, :, :]).reshape(-1, 3)
    w = np.tile(wts, cells.shape[0]) / np.prod(n)
    r = (u / n) @ lat
    phi = bloch.eval_bloch_v(beta, lat, s.k, r)[:, 0]
    for j in range(0, s.n_g, 3):
        comp = np.sum(w * phi * np.exp(-1j * r @ (s.gvecs[j] + s.k)))
        assert abs(comp - s.coef[0, j]) < 1e-11 * np.abs(s.coef).max(), (j, comp, s.coef[0, j])


# ---------------------------------------------------------------- workloads of the variants
def test_bloch_and_gradient_grid_samples_equal_planewave_sums():
    for key in (0, 6):
        s = config(key).system
        idx = np.random.default_rng(65).integers(0, np.array(s.grid), size=(40, 3))
        r = (idx / np.array(s.grid)) @ s.lattice
        f, gr, w = s.grid_values(), s.grid_gradient(), s.grid_laplacian()
        pick = lambda a: a[..., idx[:, 0], idx[:, 1], idx[:, 2], :]
        if s.bloch:
            v, g, l = bloch.pw_bloch_vgl(s.gvecs, s.coef, s.k, r)
            e = np.exp(-1j * r @ s.k)[:, None]           # samples hold periodic parts
            v, g, l = e * v, e[:, None, :] * g, e * l
        else:
            v, g, l = pw.pw_vgl(s.gvecs, s.coef, r)
        np.testing.assert_allclose(pick(f), v, atol=1e-12 * np.abs(v).max())
        np.testing.assert_allclose(np.moveaxis(pick(gr), 0, 1), g, atol=1e-12 * np.abs(g).max())
        np.testing.assert_allclose(pick(w), l, atol=1e-12 * np.abs(l).max())
    assert config(6).system.nyquist_ok() and config(7).system.nyquist_ok()
    assert np.all(np.linalg.norm(config(6).system.qvecs, axis=1) < 4.0)


# ---------------------------------------------------------------- pp-spline form
from oracle import ppspline


def _golden_pp():
    basis, centred = {}, {}
    with open(os.path.join(GOLDEN, "ppspline_basis_paper.txt")) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "basis":
                basis[(int(f[1]), int(f[2]))] = [float(Fraction(x)) for x in f[3:]]
            elif f[0] == "centred":
                centred[int(f[1])] = [float(Fraction(x)) for x in f[2:]]
    return basis, centred


def test_pp_basis_matches_printed_polynomials_and_centred_form():
    basis, centred = _golden_pp()
    t = np.linspace(0.0, 0.999, 101)
    w = ppspline.basis(t)
    for (i, kappa), c in basis.items():
        np.testing.assert_allclose(w[:, i, kappa - 1], np.polyval(c, t), atol=1e-15)
        # grid-centred picture: corner i sits at xi = t - i
        np.testing.assert_allclose(w[:, i, kappa - 1], np.polyval(centred[kappa], np.abs(t - i)), atol=1e-15)
    # the value kind interpolates linearly; the derivative kind vanishes at both corners
    np.testing.assert_allclose(ppspline.basis(np.array([0.0, 1.0]))[:, :, 1], 0.0, atol=1e-16)


def test_pp_build_values_and_second_differences_of_bspline_coefficients():
    s = make_system("pp", SKEW, (9, 8, 10), 3, 2.0, 2.0, (44, 1))
    f = s.grid_values()
    sig = ppspline.build_pp(f)
    beta = build.build_interp(f)
    np.testing.assert_array_equal(sig[..., 0, :], f)
    # at a knot the cubic B-spline's weights are (1, 4, 1)/6 for the value and (1, -2, 1) for the second
    # derivative (grid units), so each sigma is the B-spline coefficients filtered along every axis by
    # one of the two: sigma^{2,1,1} = D2_x B_y B_z beta, ..., sigma^{2,2,2} = D2_x D2_y D2_z beta
    d2 = lambda a, ax: np.roll(a, 1, ax) - 2 * a + np.roll(a, -1, ax)
    bv = lambda a, ax: (np.roll(a, 1, ax) + 4 * a + np.roll(a, -1, ax)) / 6
    for kappa in (1, 2):
        for mu in (1, 2):
            for nu in (1, 2):
                ref = beta
                for ax, k in enumerate((kappa, mu, nu)):
                    ref = d2(ref, ax) if k == 2 else bv(ref, ax)
                got = sig[..., 4 * (kappa - 1) + 2 * (mu - 1) + (nu - 1), :]
                np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_pp_spline_equals_interpolating_bspline_everywhere():
    # the periodic interpolating cubic spline is unique: both forms give the same function
    for s in (make_system("pp-skew", SKEW, (9, 8, 10), 3, 2.0, 2.0, (44, 2)), config(0).system):
        f = s.grid_values()
        lf = s.grid_laplacian()
        pos = s.positions(300)
        a = ppspline.eval_pp_vgl(ppspline.build_pp(f), s.lattice, pos, lap_sigma=ppspline.build_pp(lf))
        b = evaluate.eval_vgl(build.build_interp(f), s.lattice, pos, lap_beta=build.build_interp(lf))
        for x, y in zip(a, b):
            np.testing.assert_allclose(x, y, atol=1e-11 * np.abs(y).max())
        dflt = ppspline.eval_pp_vgl(ppspline.build_pp(f), s.lattice, pos)[2]
        np.testing.assert_allclose(dflt, evaluate.eval_vgl(build.build_interp(f), s.lattice, pos)[2],
                                   atol=1e-11 * np.abs(dflt).max())
