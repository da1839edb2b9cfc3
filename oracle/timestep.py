"""Crank-Nicolson / Adams-Bashforth and Guermond time steps of the
Navier-Stokes equations as generalized Stokes / Oseen problems (oracle).

Follows the paper's section on temporal discretization, equation GS: with
sigma = 2 / dt,
    sigma u^{n+1} - nu Lap u^{n+1} + grad p^{n+1} = f_GS,  div u^{n+1} = 0,
where the scheme's Crank-Nicolson averages of Lap u and grad p and the
Adams-Bashforth extrapolation of the convective term give, after the whole
step equation is multiplied by 2 (which is what makes the implicit side
sigma u - nu Lap u + grad p),
    f_GS = 2 f(t_{n+1/2}) + sigma u^n + nu Lap u^n - grad p^n
           - 3 (u^n . grad) u^n + (u^{n-1} . grad) u^{n-1},
and, for the first step, 2 (u^0 . grad) u^0 in place of the last two terms
(the paper's footnote).  The paper prints f(t_{n+1/2}) without the factor 2
that multiplies every other term; the factor is kept here.

In weak form with the discrete operator K = [[sigma M + A_nu, -B], [B^T, 0]]
(A_nu: viscous and Nitsche terms) the velocity load is
    F_u = F2 - (K U^n)_u + 2 sigma M u^n - 3 N(u^n) + N(u^{n-1}),
    N(w)_i = (N_i, (w . grad) w),
with F2 the load of 2 f(t_{n+1/2}); the pressure load is zero.  Every
integral is Gauss quadrature with k+3 points per direction per element.
"""
import numpy as np

from .assemble import quadrature, tensor_eval, tensor_points, tensor_weights


def _field(disc, U, pts):
    """Velocity values (npts, d) and gradients (npts, d, d) [:, c, j] = d u_c / d x_j."""
    d = disc.d
    npts = int(np.prod([len(p) for p in pts]))
    val = np.zeros((npts, d))
    grad = np.zeros((npts, d, d))
    for c, blk in enumerate(disc.vel):
        u = U[disc.offsets[c]:disc.offsets[c + 1]]
        val[:, c] = tensor_eval(disc, blk, pts) @ u
        for j in range(d):
            grad[:, c, j] = tensor_eval(disc, blk, pts, deriv_dir=j) @ u
    return val, grad


def convective_load(disc, W):
    """N(w)_i = integral of N_i . (w . grad) w for the discrete velocity W."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    val, grad = _field(disc, W, pts)
    conv = np.einsum("nj,ncj->nc", val, grad)
    return _load(disc, pts, w, conv)


def _load(disc, pts, w, g):
    """[integral of N_i g_c]_i over the velocity blocks, pressure rows 0."""
    parts = [tensor_eval(disc, blk, pts).T @ (w * g[:, c]) for c, blk in enumerate(disc.vel)]
    parts.append(np.zeros(disc.n_q))
    return np.concatenate(parts)


def cnab_rhs(disc, K, sigma, F2, U, Uold=None):
    """Load vector of the CN/AB step from U^n (and U^{n-1}; None at the first
    step): F2 - K U^n on the velocity rows, plus the quadrature load of
    2 sigma u^n - 3 (u^n . grad) u^n + (u^{n-1} . grad) u^{n-1}
    (first step: 2 sigma u^n - 2 (u^n . grad) u^n); pressure rows zero."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    v, gr = _field(disc, U, pts)
    g = 2.0 * sigma * v
    if Uold is None:
        g = g - 2.0 * np.einsum("nj,ncj->nc", v, gr)
    else:
        vo, gro = _field(disc, Uold, pts)
        g = g - 3.0 * np.einsum("nj,ncj->nc", v, gr) + np.einsum("nj,ncj->nc", vo, gro)
    out = _load(disc, pts, w, g)
    r = F2 - K @ U
    nv = disc.n_v
    out[:nv] += r[:nv]
    return out


def field_advection(disc, coeffs, c=1.0):
    """Advection a = c w for the discrete velocity field w (coefficients of
    ``disc``'s velocity space), as the callable ``assemble`` takes: it
    evaluates the field at the quadrature grid that ``assemble`` passes."""
    pts, _ = quadrature(disc)
    Xq = tensor_points(pts)

    def a(X):
        assert X.shape == Xq.shape and np.allclose(X, Xq), "field advection is evaluated at the quadrature grid"
        return c * _field(disc, coeffs, pts)[0]
    return a


def go_rhs(disc, K, sigma, F2, U):
    """Load of Guermond's step (equation GO, the step doubled): the operator
    K = K(a) advects with a^{n+1} = 3/2 u^n - 1/2 u^{n-1}, and the velocity
    load is F2 - (K U^n)_u + (N_i, 2 sigma u^n); pressure rows zero."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    v, _ = _field(disc, U, pts)
    out = _load(disc, pts, w, 2.0 * sigma * v)
    r = F2 - K @ U
    out[:disc.n_v] += r[:disc.n_v]
    return out
