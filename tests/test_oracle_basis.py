"""Pins of the oracle's 1-D basis and quadrature against closed forms."""
import math

import numpy as np
import pytest

from oracle.basis import gll_points, gauss_points, lagrange_eval, lagrange_deriv

GLL_CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_closed_forms(p):
    x, w = gll_points(p)
    xe, we = GLL_CLOSED[p]
    np.testing.assert_allclose(x, xe, atol=1e-15)
    np.testing.assert_allclose(w, we, rtol=1e-14)


@pytest.mark.parametrize("p", [2, 5, 8, 10])
def test_gll_exactness(p):
    # GLL with p+1 points integrates polynomials of degree <= 2p-1 exactly
    x, w = gll_points(p)
    for m in range(2 * p):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-13
    assert np.all(np.diff(x) > 0)


def test_gauss_closed_forms():
    x, w = gauss_points(2)
    np.testing.assert_allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    np.testing.assert_allclose(w, [1, 1], atol=1e-15)
    x, w = gauss_points(3)
    np.testing.assert_allclose(x, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-15)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("m", [3, 6, 12])
def test_gauss_exactness(m):
    x, w = gauss_points(m)
    for k in range(2 * m):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", [1, 3, 6])
def test_lagrange_interpolation_and_derivative(p):
    nodes, _ = gll_points(p)
    L = lagrange_eval(nodes, nodes)
    np.testing.assert_allclose(L, np.eye(p + 1), atol=1e-14)
    xs = np.linspace(-1, 1, 17)
    L = lagrange_eval(nodes, xs)
    D = lagrange_deriv(nodes, xs)
    np.testing.assert_allclose(L.sum(axis=0), 1.0, atol=1e-13)
    np.testing.assert_allclose(D.sum(axis=0), 0.0, atol=1e-11)
    # reproduces x^m and its derivative m x^(m-1) for m <= p
    for m in range(p + 1):
        np.testing.assert_allclose(nodes ** m @ L, xs ** m, atol=1e-12)
        dm = m * xs ** (m - 1) if m else np.zeros_like(xs)
        np.testing.assert_allclose(nodes ** m @ D, dm, atol=1e-10)
