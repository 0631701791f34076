"""Smoothing (Fourier-matched) B-spline coefficients (App. A, "Smoothing B-spline coefficients").

beta_lmn = sum_G (c_G / gamma_G) exp(i G . r_lmn),   r_lmn = a (l/N1, m/N2, n/N3),

with gamma_G the Fourier transform of one tensor-product basis function at G.
Per axis m, with theta_m = G . a_m / N_m = 2 pi n_m / N_m (the phase of G over one
grid step), the paper's three equivalent forms read
    3 [3 - 4 cos theta + cos 2 theta] / theta^4 = 24 sin^4(theta/2) / theta^4
    = (3/2) sinc^4(theta/2)
for its C = 3/2 basis, and gamma_G is the product over the three axes.  The
printed equation puts the prefactors outside the product; they belong to each
axis (each axis' basis carries its own factor C).  For the standard
normalization used here each axis' factor is (2/3) of the above, i.e.
sinc^4(theta/2), equal to 1 at theta = 0.

Dividing by gamma (rather than multiplying) makes the fundamental Fourier
components of the spline equal c_G exactly; aliases at theta + 2 pi k remain.
"""
import numpy as np


def gamma_axis(theta):
    """(2/3) * 24 sin^4(theta/2) / theta^4 (the paper's second printed form), with its limit 1 at
    theta = 0.  The first form, 3 [3 - 4 cos theta + cos 2 theta] / theta^4, is the same number
    (3 - 4 cos theta + cos 2 theta = 8 sin^4(theta/2)) but its numerator cancels: about
    1e-16 / theta^4 relative error, 1e-10 for the first harmonic of a 200-point axis."""
    theta = np.asarray(theta, dtype=np.float64)
    safe = np.where(theta == 0.0, 1.0, theta)
    val = (2.0 / 3.0) * 24.0 * (np.sin(0.5 * safe) / safe) ** 4
    return np.where(theta == 0.0, 1.0, val)


def gamma(miller, grid):
    theta = 2.0 * np.pi * np.asarray(miller, dtype=np.float64) / np.asarray(grid, dtype=np.float64)
    return gamma_axis(theta[:, 0]) * gamma_axis(theta[:, 1]) * gamma_axis(theta[:, 2])


def build_smoothing(miller, coef, grid, keep_complex=False):
    """beta [N1][N2][N3][O] from planewave coefficients coef [O, N_G] at Miller indices miller [N_G, 3].

    The real part is returned (real orbitals), or the complex coefficients with keep_complex
    (the periodic part of a Bloch orbital).  Requires each Miller index to land in its own FFT
    bin (N_i > 2 max |n_i|).
    """
    grid = tuple(int(v) for v in grid)
    miller = np.asarray(miller)
    bins = miller % np.array(grid)
    if len({tuple(x) for x in bins.tolist()}) != miller.shape[0]:
        raise ValueError("grid too coarse: two planewaves share a Fourier bin")
    scaled = np.asarray(coef, dtype=np.complex128) / gamma(miller, grid)[None, :]
    n_orb = scaled.shape[0]
    spec = np.zeros((n_orb,) + grid, dtype=np.complex128)
    spec[:, bins[:, 0], bins[:, 1], bins[:, 2]] = scaled
    total = grid[0] * grid[1] * grid[2]
    beta = np.fft.ifftn(spec, axes=(1, 2, 3)) * total
    return np.ascontiguousarray(np.moveaxis(beta if keep_complex else beta.real, 0, -1))
