"""1D B-spline bases (oracle, test infrastructure only).

The paper discretises H0(curl) with the curl-conforming multipatch IGA space
of its prior work (Section 2, Eq. discrMS).  Per patch and direction this
needs two 1D bases on an open uniform knot vector with ``n_el`` elements:

* N_{i,p}, the degree-p B-splines (Cox-de Boor recursion), i = 0..n-1 with
  n = n_el + p;
* D_i = p / (t_{i+p+1} - t_{i+1}) * N_{i+1,p-1}, i = 0..n-2, the derived
  degree-(p-1) splines, normalised so that
  d/dx sum_i c_i N_i = sum_i (c_{i+1} - c_i) D_i.

With this normalisation the discrete gradient is the signed node-to-edge
incidence matrix of the control mesh, which is what makes DOFs correspond to
control-mesh edges and lets the tree-cotree gauge of Section 3 act on edges.
"""
from __future__ import annotations

import numpy as np


def open_knots(p: int, n_el: int) -> np.ndarray:
    """Open uniform knot vector on [0, 1] with n_el elements, degree p."""
    inner = np.linspace(0.0, 1.0, n_el + 1)
    return np.concatenate([np.zeros(p), inner, np.ones(p)])


def bspline_basis(t: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """All degree-p B-splines on knots t at points x, shape (len(x), n).

    Cox-de Boor recursion with the convention 0/0 = 0.  Degree-0 functions
    use half-open intervals; the right end of the knot span is assigned to
    the last non-empty interval so the basis is a partition of unity on the
    closed interval.
    """
    t = np.asarray(t, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(t) - 1  # number of degree-0 intervals
    N = np.zeros((len(x), m))
    for i in range(m):
        if t[i] < t[i + 1]:
            N[:, i] = (t[i] <= x) & (x < t[i + 1])
    last = max(i for i in range(m) if t[i] < t[i + 1])
    N[x == t[-1], last] = 1.0
    for q in range(1, p + 1):
        Nn = np.zeros((len(x), m - q))
        for i in range(m - q):
            d1 = t[i + q] - t[i]
            d2 = t[i + q + 1] - t[i + 1]
            if d1 > 0:
                Nn[:, i] += (x - t[i]) / d1 * N[:, i]
            if d2 > 0:
                Nn[:, i] += (t[i + q + 1] - x) / d2 * N[:, i + 1]
        N = Nn
    return N


def dspline_basis(t: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """Derived splines D_i = p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}, shape (len(x), n-1)."""
    t = np.asarray(t, dtype=np.float64)
    n = len(t) - p - 1
    Nlow = bspline_basis(t, p - 1, x)  # degree p-1 functions on the same knots: n+1 of them
    D = np.zeros((Nlow.shape[0], n - 1))
    for i in range(n - 1):
        D[:, i] = p / (t[i + p + 1] - t[i + 1]) * Nlow[:, i + 1]
    return D


def bspline_deriv(t: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """First derivatives of the degree-p B-splines, shape (len(x), n).

    Textbook formula N'_{i,p} = p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}.
    """
    t = np.asarray(t, dtype=np.float64)
    n = len(t) - p - 1
    Nlow = bspline_basis(t, p - 1, x)
    dN = np.zeros((Nlow.shape[0], n))
    for i in range(n):
        a = t[i + p] - t[i]
        b = t[i + p + 1] - t[i + 1]
        if a > 0:
            dN[:, i] += p / a * Nlow[:, i]
        if b > 0:
            dN[:, i] -= p / b * Nlow[:, i + 1]
    return dN


def greville(t: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae (t_{i+1} + ... + t_{i+p}) / p."""
    n = len(t) - p - 1
    return np.array([np.mean(t[i + 1:i + p + 1]) for i in range(n)])


def gauss_legendre(nq: int):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def element_quadrature(p: int, n_el: int, nq: int):
    """Quadrature points of all elements of an open uniform knot vector.

    Returns (points (n_el*nq,), weights (n_el*nq,), element index per point).
    """
    xq, wq = gauss_legendre(nq)
    h = 1.0 / n_el
    pts = (np.arange(n_el)[:, None] + xq[None, :]) * h
    wts = np.broadcast_to(wq[None, :] * h, (n_el, nq))
    el = np.repeat(np.arange(n_el), nq)
    return pts.ravel(), wts.ravel().copy(), el
