"""Univariate B-splines for the oracle (test infrastructure only).

Follows the paper's section on univariate and multivariate B-splines: open
knot vectors whose first and last knots are repeated degree+1 times, basis
functions from the Cox-de Boor recursion, and maximal continuity on uniform
knots (stated at the start of the numerical-results section).
"""
import numpy as np
from numpy.polynomial.legendre import leggauss


def open_knots(n_elem, degree):
    """Open uniform knot vector of ``degree`` on ``n_elem`` equal elements of [0,1].

    The first and last knots are repeated degree+1 times and every interior
    knot 1/N, ..., (N-1)/N appears once (maximal continuity).  The space has
    n_elem + degree functions.
    """
    inner = np.arange(1, n_elem, dtype=np.float64) / n_elem
    return np.concatenate([np.zeros(degree + 1), inner, np.ones(degree + 1)])


def basis(knots, degree, x):
    """Values of all B-splines of ``degree`` on ``knots`` at points ``x``.

    Cox-de Boor recursion exactly as defined in the paper: degree 0 is the
    indicator of the half-open knot span [xi_i, xi_{i+1}); degree p combines
    two degree p-1 functions with the ratios (x - xi_i)/(xi_{i+p} - xi_i) and
    (xi_{i+p+1} - x)/(xi_{i+p+1} - xi_{i+1}), where a ratio with a zero
    denominator is dropped.  The right end point x = 1 is assigned to the last
    non-empty span so that the basis stays a partition of unity on [0, 1].

    Returns an array of shape (len(x), len(knots) - degree - 1).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(knots) - 1
    B = np.zeros((x.size, m))
    last = max(i for i in range(m) if knots[i + 1] > knots[i])
    for i in range(m):
        lo, hi = knots[i], knots[i + 1]
        if hi > lo:
            B[:, i] = ((x >= lo) & (x < hi)).astype(np.float64)
    B[x == knots[-1], :] = 0.0
    B[x == knots[-1], last] = 1.0
    for p in range(1, degree + 1):
        nf = m - p
        Bn = np.zeros((x.size, nf))
        for i in range(nf):
            d1 = knots[i + p] - knots[i]
            d2 = knots[i + p + 1] - knots[i + 1]
            if d1 > 0:
                Bn[:, i] += (x - knots[i]) / d1 * B[:, i]
            if d2 > 0:
                Bn[:, i] += (knots[i + p + 1] - x) / d2 * B[:, i + 1]
        B = Bn
    return B


def basis_deriv(knots, degree, x):
    """First derivatives of all B-splines of ``degree`` on ``knots`` at ``x``.

    Uses the textbook derivative of the Cox-de Boor recursion,
    N'_{i,p} = p/(xi_{i+p}-xi_i) N_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) N_{i+1,p-1},
    with the degree p-1 functions on the same knot vector and 0/0 := 0.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(knots) - degree - 1
    if degree == 0:
        return np.zeros((x.size, n))
    lower = basis(knots, degree - 1, x)
    D = np.zeros((x.size, n))
    for i in range(n):
        d1 = knots[i + degree] - knots[i]
        d2 = knots[i + degree + 1] - knots[i + 1]
        if d1 > 0:
            D[:, i] += degree / d1 * lower[:, i]
        if d2 > 0:
            D[:, i] -= degree / d2 * lower[:, i + 1]
    return D


def support(knots, degree, i):
    """Closed support [xi_i, xi_{i+degree+1}] of function i."""
    return knots[i], knots[i + degree + 1]


def gauss_rule(n_elem, npts):
    """Gauss-Legendre points and weights, ``npts`` per element, on [0,1] split
    into ``n_elem`` equal elements.  Returns (x, w) of length n_elem*npts."""
    t, wt = leggauss(npts)
    h = 1.0 / n_elem
    e = np.arange(n_elem, dtype=np.float64)[:, None]
    x = (e + 0.5 * (t[None, :] + 1.0)) * h
    w = np.broadcast_to(0.5 * h * wt[None, :], x.shape)
    return x.ravel(), np.ascontiguousarray(w).ravel()
