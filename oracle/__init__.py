"""FP64 CPU oracle for periodic tricubic B-spline orbital evaluation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants) and imports nothing
from it; the library must never call into it.

Plain numpy in float64, written for a reader to check against the paper by eye:

  pw         planewave orbital, gradient and Laplacian by direct summation
             (Sec. I, Eq. pw_orbital)
  bspline    cubic B-spline basis and its derivatives (App. A, B-splines:
             Eq. b-splinebasis and Eq. bsplinegridcenteredbasis)
  build      interpolating coefficients: the periodic tridiagonal-with-corners
             system solved one axis after the other (App. A, Interpolating
             B-spline coefficients)
  evaluate   reduced coordinates (Sec. II, Eq. reducedcoordinate), tensor-product
             evaluation (Eq. b-splineapproximation) and the chain rule back to
             Cartesian derivatives (Sec. II, Coordinates paragraph)
  adjoint    transpose of the evaluation: gradients of a scalar loss with respect
             to the coefficients and to the positions
  quantize   FP64 -> FP32 -> BF16 round-to-nearest-even storage casts
  smoothing  Fourier-matched (smoothing) B-spline coefficients (App. A,
             Eq. b-splinecoefficients)
  fit        weighted least-squares misfit with a second-difference penalty
  projection closed-form L2 projection onto the spline space: the limit of
             that fit with values only, no penalty and dense points
  lagrange   cubic Lagrange interpolation of grid values (App. A, Lagrange
             interpolation)
  separate   value, gradient and Laplacian from five separate interpolants
             (direct approximations of the derivatives, Sec. III A, Fig. 1)
  bloch      Bloch orbitals e^{ik.r} u(r): planewave sums and the product rule
             over a complex periodic interpolant (Sec. I)
  ppspline   piecewise-polynomial form of the interpolating cubic spline: 8
             numbers per grid point, 2x2x2 corners per point (App. A,
             Piecewise-polynomial-form splines)

Basis normalization: the paper scales the cubic B-spline so that its maximum is
1 (C = 3/2 in the recurrence of App. A); this oracle uses the standard
normalization (the paper's basis times 2/3), whose 64 tensor weights sum to 1.
The spline *function* is the same either way; only the stored coefficients
differ, by the constant factor (3/2)^3.
"""
from . import bspline, pw, build, evaluate, adjoint, quantize, smoothing, fit  # noqa: F401
from . import lagrange, separate, bloch, ppspline, projection  # noqa: F401
