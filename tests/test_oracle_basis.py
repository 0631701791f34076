"""Pins of the oracle's cubic B-spline basis (App. A, Eq. b-splinebasis / bsplinegridcenteredbasis)."""
import os
from fractions import Fraction

import numpy as np

from oracle import bspline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_polynomials():
    rows = {}
    with open(os.path.join(GOLDEN, "bspline_basis_paper.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[int(parts[0])] = [float(Fraction(p)) for p in parts[1:]]
    return rows


T = np.linspace(0.0, 1.0, 257, endpoint=False)


def test_grid_centred_form_matches_printed_polynomials():
    polys = paper_polynomials()
    assert sorted(polys) == [-1, 0, 1, 2]
    for k, l in enumerate((-1, 0, 1, 2)):
        printed = np.polyval(polys[l], T)
        ours = bspline.weights(T, 0)[:, k] * bspline.PAPER_C
        np.testing.assert_allclose(ours, printed, rtol=0, atol=1e-15)


def test_derivatives_match_printed_polynomials():
    polys = paper_polynomials()
    for k, l in enumerate((-1, 0, 1, 2)):
        p = np.array(polys[l])
        for order in (1, 2, 3):
            p = np.polyder(p)
            printed = np.polyval(p, T)
            ours = bspline.weights(T, order)[:, k] * bspline.PAPER_C
            np.testing.assert_allclose(ours, printed, rtol=0, atol=1e-14)


def test_partition_of_unity_standard_normalization():
    for order, expect in ((0, 1.0), (1, 0.0), (2, 0.0), (3, 0.0)):
        s = bspline.weights(T, order).sum(axis=1)
        np.testing.assert_allclose(s, expect, atol=1e-15)
    # the paper's normalization sums to 3/2 instead (C = 3/2)
    np.testing.assert_allclose(bspline.b_paper(T[:, None] - bspline.OFFSETS).sum(axis=1), 1.5, atol=1e-15)


def test_64_weights_sum_to_one():
    rng = np.random.default_rng(0)
    t = rng.random((100, 3))
    w = [bspline.weights(t[:, d]) for d in range(3)]
    tot = np.einsum("pl,pm,pn->p", *w)
    np.testing.assert_allclose(tot, 1.0, atol=1e-15)


def test_knot_values_and_support():
    assert bspline.b(0.0) == 2.0 / 3.0
    assert bspline.b(1.0) == 1.0 / 6.0 and bspline.b(-1.0) == 1.0 / 6.0
    assert bspline.b(2.0) == 0.0 and bspline.b(-2.5) == 0.0
    # continuity of value, slope and curvature across the knots xi = +-1 (C^2 basis)
    for x in (-1.0, 1.0):
        e = 1e-9
        for f in (bspline.b, bspline.db, bspline.d2b):
            assert abs(f(x - e) - f(x + e)) < 1e-8


def test_third_derivative_piecewise_constant():
    np.testing.assert_array_equal(bspline.weights(np.array([0.0, 0.3, 0.999]), 3),
                                  np.tile([-1.0, 3.0, -3.0, 1.0], (3, 1)))


def test_derivatives_finite_difference():
    xi = np.linspace(-2.2, 2.2, 97) + 1e-3     # avoid landing on the knots
    h = 1e-6
    np.testing.assert_allclose(bspline.db(xi), (bspline.b(xi + h) - bspline.b(xi - h)) / (2 * h), atol=1e-8)
    np.testing.assert_allclose(bspline.d2b(xi), (bspline.db(xi + h) - bspline.db(xi - h)) / (2 * h), atol=1e-8)
