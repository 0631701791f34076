"""Orbital value, gradient and Laplacian from five separate interpolants (Sec. III A and Fig. 1:
direct approximations of the gradient and of the Laplacian rather than derivatives of the
orbital's interpolant).

The five tables hold, in order, the orbital, the three Cartesian components of its gradient and
its Laplacian.  Each is evaluated by value only, with the basis of the representation: cubic
B-spline coefficients (App. A, Eq. b-splineapproximation) or Lagrange grid values (App. A,
Eq. lagrangeinterpolation3).  No chain rule is involved: the tables are Cartesian already.
"""
import numpy as np

from . import evaluate, lagrange


def eval_separate(tables, lattice, pos, basis="bspline"):
    """tables: sequence of 5 arrays [N1][N2][N3][O] (V, d/dx, d/dy, d/dz, Laplacian).
    Returns V [P,O], grad [P,3,O], lap [P,O]."""
    if len(tables) != 5:
        raise ValueError("five tables expected: V, three gradient components, Laplacian")
    value = evaluate.eval_v if basis == "bspline" else lagrange.eval_values
    if basis not in ("bspline", "lagrange"):
        raise ValueError(basis)
    out = [value(t, lattice, pos) for t in tables]
    return out[0], np.stack(out[1:4], axis=1), out[4]
