"""Pins of the oracle's storage casts and smoothing build, and of the seeded workloads."""
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import quantize, smoothing, evaluate, pw
from workloads import config, batched_systems, make_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- storage casts
def test_bf16_cast_matches_torch():
    rng = np.random.default_rng(30)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 65504.0, 1e-40, -3.0e38]])
    ours = quantize.to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7 in bf16: rounds to even (1.0)
    vals = np.array([1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -(1.0 + 2.0**-8)], dtype=np.float32)
    out = quantize.bf16_bits_to_f64(quantize.f32_to_bf16_bits(vals))
    np.testing.assert_array_equal(out, [1.0, 1.0 + 2 * 2.0**-7, -1.0])


def test_quantized_error_bounds():
    x = np.random.default_rng(31).standard_normal(10000)
    assert np.all(np.abs(quantize.quantized(x, "f32") - x) <= 2.0**-24 * np.abs(x))
    assert np.all(np.abs(quantize.quantized(x, "bf16") - x) <= (2.0**-8 + 2.0**-24) * np.abs(x))


# ---------------------------------------------------------------- smoothing build
def _gamma_forms(theta):
    f1 = 3 * (3 - 4 * np.cos(theta) + np.cos(2 * theta)) / theta**4
    f2 = 24 * (np.sin(theta / 2) / theta) ** 4
    f3 = 1.5 * (np.sin(theta / 2) / (theta / 2)) ** 4
    return f1, f2, f3


def test_gamma_printed_forms_agree_and_limit():
    theta = np.linspace(0.05, np.pi, 50)
    f1, f2, f3 = _gamma_forms(theta)
    np.testing.assert_allclose(f1, f2, rtol=1e-9)
    np.testing.assert_allclose(f2, f3, rtol=1e-12)
    lim = None
    with open(os.path.join(GOLDEN, "gamma_forms_paper.txt")) as fh:
        for line in fh:
            if line.startswith("limit"):
                lim = float(Fraction(line.split()[1]))
    assert abs(_gamma_forms(np.array([1e-3]))[2][0] - lim) < 1e-6
    # the oracle's per-axis gamma is the paper's scaled to the standard basis (factor 2/3)
    np.testing.assert_allclose(smoothing.gamma_axis(theta), f3 / 1.5, rtol=1e-9)
    assert smoothing.gamma_axis(np.array([0.0]))[0] == 1.0


def test_gamma_accurate_for_long_axes():
    """First harmonics of long axes (theta = 2 pi / N, N up to 1024): gamma_axis against the Taylor
    series of sinc^4(theta/2), sinc(x) = sum_k (-1)^k x^2k / (2k+1)!, to rounding."""
    from math import factorial
    for n in (24, 96, 200, 1024):
        theta = 2.0 * np.pi / n
        x = theta / 2.0
        sinc = sum((-1) ** k * x ** (2 * k) / factorial(2 * k + 1) for k in range(8))
        assert abs(smoothing.gamma_axis(np.array([theta]))[0] - sinc ** 4) <= 2e-15   # the cos form: 2e-14 at N = 24


def test_smoothing_fourier_components_match_planewave():
    # fundamental Fourier component of the smoothing spline at G, by Gauss-Legendre quadrature of
    # phi(r) exp(-i G.r) over the cell (exact to rounding: smooth integrand per grid cell)
    lat = np.diag([5.0, 5.5, 6.0])
    grid = (8, 8, 8)
    s = make_system("smooth", lat, grid, 1, 2.6, 2.0, (7, 7))
    assert s.nyquist_ok()
    beta = smoothing.build_smoothing(s.miller, s.coef, grid)
    xg, wg = np.polynomial.legendre.leggauss(10)
    xg = (xg + 1) / 2
    wg = wg / 2
    n = np.array(grid)
    cells = np.stack(np.meshgrid(*[np.arange(k) for k in grid], indexing="ij"), -1).reshape(-1, 3)
    nodes = np.stack(np.meshgrid(xg, xg, xg, indexing="ij"), -1).reshape(-1, 3)
    wts = np.einsum("i,j,k->ijk", wg, wg, wg).reshape(-1)
    u = (cells[:, None, :] + nodes[None, :, :]).reshape(-1, 3)
    w = np.tile(wts, cells.shape[0]) / np.prod(n)
    r = (u / n) @ lat
    phi = evaluate.eval_v(beta, lat, r)[:, 0]
    for j in range(0, s.n_g, 5):
        comp = np.sum(w * phi * np.exp(-1j * r @ s.gvecs[j]))
        assert abs(comp - s.coef[0, j]) < 1e-11 * np.abs(s.coef).max(), (j, comp, s.coef[0, j])


def test_smoothing_closer_to_planewave_than_interpolating():
    from oracle import build
    w = config(0)
    s = w.system
    pos = w.positions()[:400]
    vp, gp, lp = pw.pw_vgl(s.gvecs, s.coef, pos)
    bi = build.build_interp(s.grid_values())
    bs = smoothing.build_smoothing(s.miller, s.coef, s.grid)
    ei = [np.abs(a - b).mean() / np.abs(b).mean() for a, b in zip(evaluate.eval_vgl(bi, s.lattice, pos), (vp, gp, lp))]
    es = [np.abs(a - b).mean() / np.abs(b).mean() for a, b in zip(evaluate.eval_vgl(bs, s.lattice, pos), (vp, gp, lp))]
    assert es[0] < ei[0] and es[1] < ei[1], (es, ei)


# ---------------------------------------------------------------- workloads
def test_workload_counts_and_determinism():
    assert config(0).system.n_g == 283
    assert config(1).system.n_g == 9315
    a, b = config(0), config(0)
    np.testing.assert_array_equal(a.system.coef, b.system.coef)
    np.testing.assert_array_equal(a.positions(), b.positions())
    for k in (0, 1, 4, 5):
        assert config(k).system.nyquist_ok()


def test_coefficients_conjugate_symmetric():
    s = config(0).system
    index = {tuple(m): i for i, m in enumerate(s.miller.tolist())}
    for i, m in enumerate(s.miller.tolist()):
        j = index[(-m[0], -m[1], -m[2])]
        np.testing.assert_array_equal(s.coef[:, j], np.conj(s.coef[:, i]))
    assert np.all(np.sort(np.linalg.norm(s.gvecs, axis=1)) < s.gcut)


def test_grid_samples_equal_planewave_sum():
    for key in (0, 5):
        s = config(key).system
        f = s.grid_values()
        lf = s.grid_laplacian()
        rng = np.random.default_rng(32)
        idx = rng.integers(0, np.array(s.grid), size=(50, 3))
        r = (idx / np.array(s.grid)) @ s.lattice
        v, _, lap = pw.pw_vgl(s.gvecs, s.coef, r)
        np.testing.assert_allclose(f[idx[:, 0], idx[:, 1], idx[:, 2]], v, atol=1e-12 * np.abs(v).max())
        np.testing.assert_allclose(lf[idx[:, 0], idx[:, 1], idx[:, 2]], lap, atol=1e-12 * np.abs(lap).max())


def test_batched_workload_shape():
    systems = batched_systems(scale=1.0)
    assert len(systems) == 48
    for w in systems:
        assert 32 <= w.system.n_orb <= 256 and 24 <= w.system.grid[0] <= 64
        assert 16 * 64 <= w.n_pts <= 512 * 256
    total = sum(w.n_pts * w.system.n_orb for w in systems)
    assert 1e8 < total < 6e8
