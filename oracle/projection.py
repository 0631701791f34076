"""L2 projection of planewave orbitals onto the periodic cubic spline space (closed form).

Test infrastructure: the limit that a least-squares fit of spline coefficients to orbital values
(no smoothness term, value misfit only, dense uniform points) tends to.  The spline is
s(u) = sum_j beta_j B(u - j) with the cubic B-spline of App. A (Eq. bsplinegridcenteredbasis,
standard normalization) and u in grid units.  Minimizing the mean of (s - f)^2 gives, per axis,
the normal equations G beta = r with a circulant Gram matrix G, so a planewave e^{i theta u}
(theta = 2 pi n / N, the phase per grid step) has coefficients

    beta = [ bhat(theta) / A(theta) ] e^{i theta j},

A the Gram symbol and bhat the Fourier transform of the basis; in 3D the factors multiply.
Two versions of the integral over the cell:
  - continuous (m=None): A(theta) = 151/315 + (397/840) cos theta + (1/21) cos 2 theta
    + (1/2520) cos 3 theta (the autocorrelation of B, the septic B-spline, at the integers)
    and bhat(theta) = sinc^4(theta / 2);
  - a lattice of m midpoints per cell and axis (m an integer): the midpoint-rule sums of the
    same two integrals, for which the closed form is the exact least-squares minimizer.
"""
import numpy as np

from .bspline import b


def gram_symbol(theta, m=None):
    theta = np.asarray(theta, dtype=np.float64)
    if m is None:
        return (151 / 315 + (397 / 840) * np.cos(theta) + (1 / 21) * np.cos(2 * theta)
                + (1 / 2520) * np.cos(3 * theta))
    x = (np.arange(m) + 0.5) / m
    out = np.zeros_like(theta)
    for c in range(-2, 2):                       # cells meeting the support (-2, 2) of B
        bx = b(c + x)
        for d in range(-3, 4):
            out = out + np.sum(bx * b(c + x - d)) * np.cos(d * theta)
    return out / m


def basis_symbol(theta, m=None):
    theta = np.asarray(theta, dtype=np.float64)
    if m is None:
        return (np.sinc(theta / (2 * np.pi)) ** 4).astype(np.complex128)   # sinc(x) = sin(pi x)/(pi x)
    x = (np.arange(m) + 0.5) / m
    out = np.zeros(theta.shape, dtype=np.complex128)
    for c in range(-2, 2):
        u = c + x
        out = out + np.sum(b(u) * np.exp(1j * np.multiply.outer(theta, u)), axis=-1)
    return out / m


def project(miller, coef, grid, m=None):
    """Coefficients [N1][N2][N3][O] of the projection of the real orbitals
    sum_G c_G e^{2 pi i n.s} (miller [N_G,3] integer, coef [O,N_G] with conjugate partners)."""
    miller = np.asarray(miller)
    n = np.asarray(grid)
    theta = 2 * np.pi * miller / n
    mult = np.ones(miller.shape[0], dtype=np.complex128)
    for ax in range(3):
        mult *= basis_symbol(theta[:, ax], m) / gram_symbol(theta[:, ax], m)
    spec = np.zeros((coef.shape[0],) + tuple(grid), dtype=np.complex128)
    idx = tuple((miller % n).T)
    for o in range(coef.shape[0]):
        np.add.at(spec[o], idx, coef[o] * mult)
    vals = np.fft.ifftn(spec, axes=(1, 2, 3)) * np.prod(n)
    return np.ascontiguousarray(np.moveaxis(vals.real, 0, -1))
