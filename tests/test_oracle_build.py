"""Pins of the oracle's interpolating build (App. A, Interpolating B-spline coefficients)."""
import numpy as np
import pytest

from oracle import build, evaluate
from workloads import config


def test_knot_matrix_is_periodic_tridiagonal():
    for n in (4, 5, 9, 16):
        m = build.periodic_knot_matrix(n)
        expect = np.zeros((n, n))
        for i in range(n):
            expect[i, i] = 4.0 / 6.0
            expect[i, (i + 1) % n] = 1.0 / 6.0
            expect[i, (i - 1) % n] = 1.0 / 6.0
        np.testing.assert_allclose(m, expect, atol=1e-16)


@pytest.mark.parametrize("grid", [(8, 8, 8), (5, 6, 7), (16, 12, 10)])
def test_single_planewave_closed_form(grid):
    # f_j = exp(i theta . j) is an eigenvector of each circulant with eigenvalue (4 + 2 cos theta)/6
    n = np.array(grid)
    miller = np.array([1, 2, -1])
    theta = 2 * np.pi * miller / n
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in grid], indexing="ij"), axis=-1)
    phase = idx @ theta
    f = np.stack([np.cos(phase), np.sin(phase)], axis=-1)        # two real orbitals
    lam = np.prod((4 + 2 * np.cos(theta)) / 6)
    beta = build.build_interp(f)
    np.testing.assert_allclose(beta, f / lam, atol=1e-14)


def test_matches_circulant_fft_route():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((10, 7, 12, 3))
    beta = build.build_interp(f)
    lam = [(4 + 2 * np.cos(2 * np.pi * np.arange(n) / n)) / 6 for n in f.shape[:3]]
    spec = np.fft.fftn(f, axes=(0, 1, 2)) / (lam[0][:, None, None, None] * lam[1][None, :, None, None]
                                            * lam[2][None, None, :, None])
    ref = np.fft.ifftn(spec, axes=(0, 1, 2)).real
    np.testing.assert_allclose(beta, ref, atol=1e-13)


def test_dense_kronecker_brute_force():
    rng = np.random.default_rng(2)
    grid = (4, 5, 6)
    f = rng.standard_normal(grid + (2,))
    mats = []
    for n in grid:
        m = np.zeros((n, n))
        for i in range(n):           # basis centred at l, value at knot i: 4/6 on, 1/6 off (periodic)
            m[i, i] += 4 / 6
            m[i, (i + 1) % n] += 1 / 6
            m[i, (i - 1) % n] += 1 / 6
        mats.append(m)
    big = np.kron(np.kron(mats[0], mats[1]), mats[2])
    ref = np.linalg.solve(big, f.reshape(-1, 2)).reshape(f.shape)
    np.testing.assert_allclose(build.build_interp(f), ref, atol=1e-13)


@pytest.mark.parametrize("key", [0, 5])
def test_interpolates_grid_values(key):
    w = config(key)
    s = w.system
    f = s.grid_values()
    beta = build.build_interp(f)
    n = np.array(s.grid)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, n, size=(300, 3))
    # grid point r = a (i/N); shift by a lattice vector multiple to also test the fold
    pos = (idx / n) @ s.lattice + rng.integers(-2, 3, size=(300, 1)) * s.lattice[0]
    v, _, _ = evaluate.eval_vgl(beta, s.lattice, pos)
    ref = f[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.abs(v - ref).max() <= 5e-13 * np.abs(f).max()
