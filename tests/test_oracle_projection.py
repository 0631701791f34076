"""Pins of oracle/projection.py and of the fit loss at its least-squares limit.

With no smoothness term (lambda = 0) and no Laplacian term (w_L = 0) the fit loss of
oracle/fit.py is the mean squared misfit of the spline's value at the fit points.  It is
quadratic in the coefficients, so its minimizer is where its gradient vanishes.  On a lattice of
m midpoints per cell and axis the minimizer has the closed form of oracle/projection.py (App. A,
Eq. b-splineapproximation with the basis of Eq. bsplinegridcenteredbasis), and as m grows it
tends to the continuous L2 projection (the septic-B-spline Gram symbol and sinc^4).
"""
import numpy as np

from oracle import build, fit, projection
from oracle.bspline import b

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])   # rows a_i
GRID = (6, 7, 8)


def test_septic_symbol_is_autocorrelation_of_the_basis():
    """A(theta) = sum_d (int B(x) B(x - d) dx) cos(d theta): the integrals by Gauss-Legendre
    quadrature on each unit interval (exact for these piecewise polynomials)."""
    xg, wg = np.polynomial.legendre.leggauss(8)
    theta = np.linspace(-np.pi, np.pi, 65)
    ref = np.zeros_like(theta)
    for d in range(-3, 4):
        acc = 0.0
        for c in range(-2, 2):
            x = c + 0.5 * (xg + 1)
            acc += 0.5 * np.sum(wg * b(x) * b(x - d))
        ref += acc * np.cos(d * theta)
    np.testing.assert_allclose(projection.gram_symbol(theta), ref, rtol=0, atol=1e-15)
    # and the transform of B: sinc^4(theta/2), also by quadrature
    bh = np.zeros(theta.shape, dtype=np.complex128)
    for c in range(-2, 2):
        x = c + 0.5 * (xg + 1)
        bh += 0.5 * np.sum(wg[None, :] * b(x)[None, :] * np.exp(1j * np.multiply.outer(theta, x)), axis=1)
    np.testing.assert_allclose(projection.basis_symbol(theta), bh, rtol=0, atol=1e-9)


def test_discrete_symbols_tend_to_continuous_projection():
    theta = np.linspace(-np.pi, np.pi, 257)
    errs_a, errs_b = [], []
    for m in (2, 4, 8, 16, 32, 64):
        errs_a.append(np.abs(projection.gram_symbol(theta, m) - projection.gram_symbol(theta)).max())
        errs_b.append(np.abs(projection.basis_symbol(theta, m) - projection.basis_symbol(theta)).max())
    # midpoint rule on piecewise polynomials: second order in 1/m
    for e in (errs_a, errs_b):
        ratios = np.array(e[:-1]) / np.array(e[1:])
        assert np.all(ratios > 3.5), ratios
    assert errs_a[-1] < 1e-4 and errs_b[-1] < 1e-4
    assert abs(projection.gram_symbol(0.0) - 1.0) < 1e-15          # B sums to one
    assert projection.gram_symbol(np.pi) > 0.05                     # positive definite


def _lattice_points(m):
    axes = [(np.arange(n * m) + 0.5) / m for n in GRID]       # grid units, m midpoints per cell
    u = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    return u / np.asarray(GRID)                                # crystal coordinates s


def _orbitals(rng, n_orb):
    """Real orbitals: Miller indices with |n_i| <= 2 on a half space, their conjugate partners."""
    rng_n = range(-2, 3)
    half = [(a, b_, c) for a in rng_n for b_ in rng_n for c in rng_n if (a, b_, c) > (0, 0, 0)]
    miller = np.array([(0, 0, 0)] + half + [tuple(-x for x in h) for h in half])
    k = len(half)
    coef = np.zeros((n_orb, miller.shape[0]), dtype=np.complex128)
    for o in range(n_orb):
        c = rng.standard_normal(k) + 1j * rng.standard_normal(k)
        c *= np.exp(-0.25 * np.sum(miller[1:1 + k] ** 2, axis=1))
        coef[o, 0] = rng.standard_normal()
        coef[o, 1:1 + k] = c
        coef[o, 1 + k:] = np.conj(c)
    return miller, coef


def _values(miller, coef, s):
    return np.real(np.exp(2j * np.pi * (s @ miller.T)) @ coef.T)      # [P, O]


def test_oracle_fit_minimizer_is_discrete_projection():
    m = 3
    rng = np.random.default_rng(34)
    n_orb = 2
    miller, coef = _orbitals(rng, n_orb)
    s = _lattice_points(m)
    pos = s @ SKEW
    v_t = _values(miller, coef, s)
    lap_t = np.zeros_like(v_t)
    w_v = 1.0 / np.mean(v_t * v_t)

    def loss_grad(beta):
        return fit.loss_and_grad(beta, SKEW, pos, v_t, lap_t, w_v, 0.0, 0.0)

    beta_cf = projection.project(miller, coef, GRID, m)
    loss_cf, g_cf = loss_grad(beta_cf)
    # the interpolating spline of the same orbitals (the fit's starting point)
    axes = [np.arange(n) / n for n in GRID]
    sg = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    beta_int = build.build_interp(_values(miller, coef, sg).reshape(GRID + (n_orb,)))
    loss_int, g_int = loss_grad(beta_int)
    assert np.linalg.norm(g_cf) <= 1e-11 * np.linalg.norm(g_int), (np.linalg.norm(g_cf), np.linalg.norm(g_int))
    assert loss_cf < 0.7 * loss_int
    # a positive definite quadratic: a perturbed table has a larger loss
    d = rng.standard_normal(beta_cf.shape) * 1e-3
    assert loss_grad(beta_cf + d)[0] > loss_cf
    # the continuous projection is already close to the lattice optimum at m = 3
    loss_c, _ = loss_grad(projection.project(miller, coef, GRID))
    assert loss_cf <= loss_c <= loss_cf * (1 + 1e-3)
