"""Pins of the oracle's 1D spline bases against mathematics and SciPy.

Covers the basis construction behind Section 2's curl-conforming space.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle.bspline import (bspline_basis, bspline_deriv, dspline_basis, element_quadrature,
                            gauss_legendre, greville, open_knots)

CASES = [(1, 1), (1, 3), (2, 1), (2, 4), (3, 2), (3, 8), (4, 5)]


@pytest.mark.parametrize("p,n_el", CASES)
def test_matches_scipy_bspline(p, n_el):
    t = open_knots(p, n_el)
    x = np.linspace(0, 1, 101)[:-1] + 0.003
    N = bspline_basis(t, p, x)
    n = len(t) - p - 1
    assert N.shape == (len(x), n)
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        ref = BSpline(t, c, p, extrapolate=False)(x)
        np.testing.assert_allclose(N[:, i], ref, atol=1e-14)


@pytest.mark.parametrize("p,n_el", CASES)
def test_partition_of_unity_and_greville(p, n_el):
    t = open_knots(p, n_el)
    x = np.linspace(0, 1, 57)
    N = bspline_basis(t, p, x)
    np.testing.assert_allclose(N.sum(axis=1), 1.0, atol=1e-14)
    # Marsden identity for the linear monomial: sum_i greville_i N_i(x) = x
    np.testing.assert_allclose(N @ greville(t, p), x, atol=1e-14)


@pytest.mark.parametrize("p,n_el", CASES)
def test_derivative_identity(p, n_el):
    """d/dx sum c_i N_i = sum (c_{i+1} - c_i) D_i, i.e. N'_i = D_{i-1} - D_i."""
    t = open_knots(p, n_el)
    x = np.linspace(0, 1, 77)[1:-1] + 1e-3
    dN = bspline_deriv(t, p, x)
    D = dspline_basis(t, p, x)
    Dpad = np.hstack([np.zeros((len(x), 1)), D, np.zeros((len(x), 1))])
    np.testing.assert_allclose(dN, Dpad[:, :-1] - Dpad[:, 1:], atol=1e-12)
    # derivative also against SciPy's own differentiation
    n = len(t) - p - 1
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        ref = BSpline(t, c, p).derivative()(x)
        np.testing.assert_allclose(dN[:, i], ref, atol=1e-11)


@pytest.mark.parametrize("p,n_el", CASES)
def test_dsplines_have_unit_integral(p, n_el):
    """int D_i = p/(t_{i+p+1}-t_{i+1}) * (t_{i+p+1}-t_{i+1})/p = 1."""
    t = open_knots(p, n_el)
    xq, wq, _ = element_quadrature(p, n_el, p + 1)
    D = dspline_basis(t, p, xq)
    np.testing.assert_allclose(wq @ D, 1.0, atol=1e-14)


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5])
def test_gauss_legendre_exactness(nq):
    x, w = gauss_legendre(nq)
    for deg in range(2 * nq):
        assert abs(w @ x**deg - 1.0 / (deg + 1)) < 1e-14
    deg = 2 * nq
    assert abs(w @ x**deg - 1.0 / (deg + 1)) > 1e-8


def test_linear_hats_closed_form():
    t = open_knots(1, 4)
    x = np.array([0.1, 0.3, 0.6, 0.9])
    N = bspline_basis(t, 1, x)
    h = 0.25
    for i in range(5):
        np.testing.assert_allclose(N[:, i], np.maximum(0, 1 - np.abs(x - i * h) / h), atol=1e-15)
