"""Manufactured solutions used by the oracle's load vectors and error checks.

The paper manufactures its forcing as f = sigma u - nu Lap u + grad p (Stokes)
plus a . grad u (Oseen) from a chosen divergence-free u and pressure p.  The
workloads here take u as the curl of a sin^2 potential:
  2D: psi = s(x) s(y), u = (d_y psi, -d_x psi)      (u = grad-perp of psi)
      p = sin(2 pi x) sin(2 pi y)
  3D: psi = (g, 0, g), g = s(x) s(y) s(z), u = curl psi
      p = sin(2 pi x) sin(2 pi y) sin(2 pi z)
with s(t) = sin^2(pi t).  u vanishes on the boundary and p has zero mean.
"""
import numpy as np

PI = np.pi


def _s(n, t):
    """n-th derivative of s(t) = sin^2(pi t)."""
    if n == 0:
        return np.sin(PI * t) ** 2
    if n == 1:
        return PI * np.sin(2 * PI * t)
    if n == 2:
        return 2 * PI ** 2 * np.cos(2 * PI * t)
    if n == 3:
        return -4 * PI ** 3 * np.sin(2 * PI * t)
    raise ValueError(n)


def _G(orders, X):
    out = np.ones(X.shape[0])
    for j, n in enumerate(orders):
        out = out * _s(n, X[:, j])
    return out


def _velocity_terms(d):
    """u_c as sums of coef * prod_j s^{(n_j)}(x_j)."""
    if d == 2:
        return [[(1.0, (0, 1))], [(-1.0, (1, 0))]]
    return [[(1.0, (0, 1, 0))],
            [(1.0, (0, 0, 1)), (-1.0, (1, 0, 0))],
            [(-1.0, (0, 1, 0))]]


def _eval_terms(terms, X, extra=None):
    out = np.zeros(X.shape[0])
    for coef, orders in terms:
        o = list(orders)
        if extra is not None:
            for j, n in extra:
                o[j] += n
        out += coef * _G(o, X)
    return out


def velocity(d, X):
    return np.stack([_eval_terms(t, X) for t in _velocity_terms(d)], axis=1)


def velocity_grad(d, X):
    """(n, d, d): [:, c, j] = d u_c / d x_j."""
    T = _velocity_terms(d)
    return np.stack([np.stack([_eval_terms(T[c], X, [(j, 1)]) for j in range(d)], axis=1)
                     for c in range(d)], axis=1)


def velocity_laplacian(d, X):
    T = _velocity_terms(d)
    return np.stack([sum(_eval_terms(T[c], X, [(j, 2)]) for j in range(d)) for c in range(d)], axis=1)


def pressure(d, X):
    out = np.ones(X.shape[0])
    for j in range(d):
        out = out * np.sin(2 * PI * X[:, j])
    return out


def pressure_grad(d, X):
    cols = []
    for j in range(d):
        g = np.ones(X.shape[0])
        for i in range(d):
            g = g * ((2 * PI * np.cos(2 * PI * X[:, i])) if i == j else np.sin(2 * PI * X[:, i]))
        cols.append(g)
    return np.stack(cols, axis=1)


def forcing(d, nu, sigma, advection=None):
    """f = sigma u - nu Lap u + grad p (+ (a . grad) u)."""
    def f(X):
        out = sigma * velocity(d, X) - nu * velocity_laplacian(d, X) + pressure_grad(d, X)
        if advection is not None:
            a = advection(X)
            gu = velocity_grad(d, X)
            out = out + np.einsum("nj,ncj->nc", a, gu)
        return out
    return f


def manufactured_advection(d, c):
    """Advection a = c u with u the manufactured velocity (the paper's Oseen
    problems advect with the manufactured velocity field)."""
    def a(X):
        return c * velocity(d, X)
    return a
