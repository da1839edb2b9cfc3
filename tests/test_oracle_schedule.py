"""Pins of the oracle's Chebyshev damping schedule: the dampings reproduce the
scaled Chebyshev polynomial and its minimax bound, scheduled smoothing steps
are that polynomial of the smoother's operator, a constant schedule is the
plain damped smoother, the eigenvalue of the undamped smoother's operator
agrees with an Arnoldi solver and does not depend on h, and scheduled cycles
keep the velocity divergence-free while contracting faster."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla
from numpy.polynomial import chebyshev as C

from oracle.multigrid import (Hierarchy, mgv, eta_levels, smooth, chebyshev_dampings, chebyshev_schedule,
                              smoother_matrix, lmax_dense, schwarz_correction)
from oracle.assemble import load_vector
from oracle.manufactured import forcing
from oracle.diagnostics import div_norm
from oracle.complex import random_divfree_start


@pytest.mark.parametrize("b,alpha,nu", [(9.45, 10.0, 1), (9.45, 10.0, 4), (5.0, 3.0, 6), (24.0, 30.0, 8)])
def test_dampings_give_the_scaled_chebyshev_polynomial(b, alpha, nu):
    """prod_j (1 - x eta_j) = T_nu(t(x)) / T_nu(t(0)), t(x) = (b + a - 2x)/(b - a),
    with T_nu from numpy's Chebyshev series; both orders give it."""
    a = b / alpha
    x = np.linspace(-0.2 * b, 1.2 * b, 301)
    t = lambda y: (b + a - 2 * y) / (b - a)
    ref = C.chebval(t(x), [0] * nu + [1]) / C.chebval(t(0.0), [0] * nu + [1])
    for rev in (False, True):
        eta = chebyshev_dampings(b, alpha, nu, reverse=rev)
        assert len(eta) == nu
        p = np.ones_like(x)
        for e in eta:
            p *= 1 - x * e
        np.testing.assert_allclose(p, ref, rtol=1e-10, atol=1e-12)
    assert chebyshev_dampings(b, alpha, nu, reverse=True) == chebyshev_dampings(b, alpha, nu)[::-1]


@pytest.mark.parametrize("alpha,nu", [(4.0, 2), (10.0, 4), (10.0, 6)])
def test_minimax_bound_on_the_interval(alpha, nu):
    """max over [a, b] of |p| is 1 / T_nu((b + a)/(b - a)) = 1 / cosh(nu acosh(.)),
    reached at the extrema of T_nu, and the dampings lie in [1/b, alpha/b]."""
    b = 9.0
    a = b / alpha
    eta = chebyshev_dampings(b, alpha, nu)
    x = np.linspace(a, b, 20001)
    p = np.prod([1 - x * e for e in eta], axis=0)
    bound = 1.0 / np.cosh(nu * np.arccosh((b + a) / (b - a)))
    assert abs(np.abs(p).max() - bound) <= 1e-9 * bound
    assert min(eta) >= 1 / b - 1e-15 and max(eta) <= alpha / b + 1e-15


def test_constant_schedule_is_the_damped_smoother():
    h = Hierarchy(2, 16, 2, 3, 1.0, 1.0)
    F = load_vector(h.finest.disc, forcing(2, 1.0, 1.0))
    U0 = np.zeros_like(F)
    plain = mgv(h, 2, U0, F, 3, 2, eta_levels(h, 0.2))
    sched = mgv(h, 2, U0, F, 3, 2, eta_levels(h, [((0.2,) * 3, (0.2,) * 2)] * 2))
    assert np.array_equal(plain, sched)


def test_scheduled_steps_are_the_polynomial_of_the_operator():
    """nu smoothing steps with F = 0 map U to prod_j (I - eta_j S^-1 K) U
    (dense S^-1 K of a tiny level)."""
    h = Hierarchy(2, 8, 2, 2, 1.0, 1.0)
    lv = h.levels[1]
    X = smoother_matrix(lv) @ lv.K.toarray()
    rng = np.random.default_rng(3)
    U = rng.standard_normal(lv.disc.n)
    eta = chebyshev_dampings(9.4, 10.0, 4)
    V = U.copy()
    for e in eta:
        V = smooth(lv, V, np.zeros_like(U), e)
    W = U.copy()
    for e in eta:
        W = W - e * (X @ W)
    np.testing.assert_allclose(V, W, rtol=0, atol=1e-12 * abs(W).max())
    # the dense S^-1 is the oracle's smoother applied to the unit vectors
    j = 17
    np.testing.assert_allclose(smoother_matrix(lv)[:, j], schwarz_correction(lv, np.eye(lv.disc.n)[j]), atol=1e-14)


@pytest.mark.parametrize("k", [1, 2])
def test_lmax_agrees_with_arnoldi_and_is_h_independent(k):
    vals = []
    for N in (8, 16):
        h = Hierarchy(2, N, k, 2, 1.0, 1.0)
        lv = h.levels[1]
        lam = lmax_dense(lv)
        X = sla.LinearOperator((lv.disc.n,) * 2, matvec=lambda v: schwarz_correction(lv, lv.K @ v))
        ev = sla.eigs(X, k=1, which="LM", return_eigenvectors=False, tol=1e-12, maxiter=20000)
        assert abs(abs(ev[0]) - lam) <= 1e-6 * lam  # clustered eigenvalues of a non-normal operator
        vals.append(lam)
    assert abs(vals[0] - vals[1]) <= 0.02 * vals[1]
    assert vals[1] > 1.0   # the summed local corrections overshoot on some modes


def test_scheduled_cycles_stay_divergence_free_and_contract_faster():
    h = Hierarchy(2, 16, 2, 3, 1.0, 1.0)
    disc = h.finest.disc
    F = load_vector(disc, forcing(2, 1.0, 1.0))
    rng = np.random.default_rng(5)
    U0 = random_divfree_start(disc, rng.standard_normal(disc.n_psi), rng.standard_normal(disc.n_q))
    lm = [lmax_dense(h.levels[2]), lmax_dense(h.levels[1])]
    sched = eta_levels(h, chebyshev_schedule(h, lm, 10.0, 4, 4))
    plain = eta_levels(h, 0.2)
    Us, Up = U0.copy(), U0.copy()
    for _ in range(4):
        Us = mgv(h, 2, Us, F, 4, 4, sched)
        Up = mgv(h, 2, Up, F, 4, 4, plain)
        assert div_norm(disc, Us) <= 1e-11 * max(1.0, np.linalg.norm(Us))
    rs = np.linalg.norm(F - h.finest.K @ Us)
    rp = np.linalg.norm(F - h.finest.K @ Up)
    assert rs < 0.5 * rp
