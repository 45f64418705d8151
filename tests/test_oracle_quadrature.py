"""Pins of the oracle's velocity quadrature (Section 2.2, last paragraph).

Gauss-Hermite is pinned to numpy's independent Golub-Welsch routine and to the
exact Gaussian moments; the Newton-Cotes rules to their polynomial degree of
exactness (which also identifies which composite rule was chosen).
"""
import math

import numpy as np
import pytest

from oracle import quadrature_1d


@pytest.mark.parametrize("n", [2, 5, 6, 9, 16, 28, 60])
def test_gauss_hermite_matches_library(n):
    x, W = quadrature_1d(0, n)
    xr, wr = np.polynomial.hermite.hermgauss(n)
    assert np.max(np.abs(x - xr)) <= 1e-13 * max(1.0, np.abs(xr).max())
    # the oracle's weights integrate g(x) dx, i.e. they carry exp(x^2)
    w = W * np.exp(-x ** 2)
    assert np.max(np.abs(w - wr) / wr) <= 1e-11


@pytest.mark.parametrize("n", [6, 16, 28])
def test_gauss_hermite_gaussian_moments(n):
    x, W = quadrature_1d(0, n)
    g = np.exp(-x ** 2)
    for k in range(n):  # exact for degree 2n-1
        exact = math.gamma(k + 0.5)
        assert abs(np.sum(W * g * x ** (2 * k)) - exact) <= 1e-13 * exact
        assert abs(np.sum(W * g * x ** (2 * k + 1))) <= 1e-13 * exact


def _poly_exact(deg, a):
    return 0.0 if deg % 2 else 2.0 * a ** (deg + 1) / (deg + 1)


@pytest.mark.parametrize("n,exact_deg", [(101, 5), (100, 3), (11, 3), (8, 1), (13, 5), (10, 3)])
def test_newton_cotes_degree(n, exact_deg):
    a = 3.0
    x, w = quadrature_1d(1, n, a)
    assert np.allclose(x, np.linspace(-a, a, n), rtol=0, atol=1e-14)
    for d in range(exact_deg + 1):
        ref = _poly_exact(d, a)
        assert abs(np.sum(w * x ** d) - ref) <= 1e-12 * max(1.0, abs(ref))
    # the next even degree is not exact: the rule is exactly the one intended
    d = exact_deg + 1
    assert abs(np.sum(w * x ** d) - _poly_exact(d, a)) > 1e-10


def test_newton_cotes_gaussian_range():
    # [-4, 4] in units of sqrt(2RT_ref): the truncated tail of exp(-x^2) is erfc(4) sqrt(pi)
    x, w = quadrature_1d(1, 101, 4.0)
    approx = np.sum(w * np.exp(-x ** 2))
    assert abs(approx - math.sqrt(math.pi)) < 1e-7
    assert abs(approx - math.sqrt(math.pi) * math.erf(4.0)) < 1e-9
