"""Cubic B-spline basis on a uniform grid (App. A, B-splines subsection).

The paper gives the basis in the grid-centred picture (Eq. bsplinegridcenteredbasis),
with the normalization C = 3/2 that makes its maximum equal to 1:

    b_paper(xi) = 3/4 |xi|^3 - 3/2 xi^2 + 1     for 0 <= |xi| < 1
                = 1/4 (2 - |xi|)^3                for 1 <= |xi| < 2
                = 0                               for |xi| >= 2

and b_l(t) = b(t - l) for the four grid points l = -1, 0, 1, 2 around a reduced
coordinate t in [0, 1) (Eq. b-splinebasis).  With C = 3/2 the four values sum to
3/2, so the oracle uses the standard normalization b = (2/3) b_paper, for which
the four values (and the 64 tensor-product weights) sum to exactly 1.
"""
import numpy as np

PAPER_C = 1.5                     # the paper's choice of the degree-0 constant
STD_SCALE = 1.0 / PAPER_C         # standard basis = paper basis * 2/3
OFFSETS = np.array([-1, 0, 1, 2])  # grid points around t, relative to floor(u)


def b_paper(xi):
    """Grid-centred cubic B-spline with the paper's normalization (maximum 1)."""
    a = np.abs(np.asarray(xi, dtype=np.float64))
    inner = 0.75 * a**3 - 1.5 * a**2 + 1.0
    outer = 0.25 * (2.0 - a) ** 3
    return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))


def b(xi):
    """Standard-normalized cubic B-spline, (2/3) * b_paper."""
    return STD_SCALE * b_paper(xi)


def db(xi):
    """d b / d xi of the standard basis (piecewise quadratic, continuous)."""
    x = np.asarray(xi, dtype=np.float64)
    a = np.abs(x)
    s = np.sign(x)
    # d/dxi of (2/3)(3/4 a^3 - 3/2 a^2 + 1) = (2/3)(9/4 a^2 - 3 a) * sign(xi)
    inner = STD_SCALE * (2.25 * a**2 - 3.0 * a) * s
    # d/dxi of (2/3)(1/4)(2 - a)^3 = -(2/3)(3/4)(2 - a)^2 * sign(xi)
    outer = -STD_SCALE * 0.75 * (2.0 - a) ** 2 * s
    return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))


def d2b(xi):
    """d^2 b / d xi^2 of the standard basis (piecewise linear, continuous)."""
    a = np.abs(np.asarray(xi, dtype=np.float64))
    inner = STD_SCALE * (4.5 * a - 3.0)
    outer = STD_SCALE * 1.5 * (2.0 - a)
    return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))


def d3b(xi):
    """d^3 b / d xi^3 of the standard basis (piecewise constant).

    Taken right-continuous at the knots: the value on [k, k+1) is used at xi = k.
    """
    x = np.asarray(xi, dtype=np.float64)
    # on [0,1): +3 ; on [-1,0): -3 ; on [1,2): -1 ; on [-2,-1): +1 ; else 0
    return np.where((x >= 0) & (x < 1), 3.0,
           np.where((x >= -1) & (x < 0), -3.0,
           np.where((x >= 1) & (x < 2), -1.0,
           np.where((x >= -2) & (x < -1), 1.0, 0.0)))) * STD_SCALE * 1.5


def weights(t, order=0):
    """Values of the d^order/dt^order b_l(t), l = -1..2, for t in [0, 1).

    t: array [...]; returns array [..., 4].
    """
    t = np.asarray(t, dtype=np.float64)[..., None]
    xi = t - OFFSETS
    fn = (b, db, d2b, d3b)[order]
    return fn(xi)
