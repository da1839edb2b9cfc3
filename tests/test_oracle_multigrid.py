"""Pins of the oracle's V-cycle and solver: direct-solve agreement,
divergence-free invariant, h-independent convergence."""
import numpy as np
import pytest

import workloads
from oracle.multigrid import Hierarchy, mgv, eta_levels, vcycles, solve, residual_norm, smooth
from oracle.assemble import load_vector, rotation_field
from oracle.manufactured import forcing
from oracle.diagnostics import direct_solve, div_norm, l2_norm_velocity
from oracle.complex import random_divfree_start


@pytest.mark.parametrize("d,N,k,L", [(2, 16, 1, 3), (2, 16, 2, 3), (3, 8, 1, 3)])
def test_vcycle_converges_to_direct_solution(d, N, k, L):
    h = Hierarchy(d, N, k, L, 1.0, 1.0)
    disc = h.finest.disc
    F = load_vector(disc, forcing(d, 1.0, 1.0))
    U, hist = solve(h, F, tol=1e-13, max_cycles=400)
    Ud = direct_solve(disc, h.finest.K, F)
    nv = disc.n_v
    assert np.linalg.norm(U[:nv] - Ud[:nv]) <= 1e-10 * np.linalg.norm(Ud[:nv])
    np.testing.assert_allclose(U[nv:], Ud[nv:], atol=1e-9 * abs(Ud[nv:]).max())


def test_coarse_solve_is_exact_with_zero_mean_pressure():
    h = Hierarchy(2, 8, 2, 2, 1.0, 1.0)
    lv = h.levels[0]
    rng = np.random.default_rng(0)
    G = rng.standard_normal(lv.disc.n)
    G[lv.disc.n_v:] -= G[lv.disc.n_v:].mean()      # consistent: sum of pressure rows is 0
    x = lv.coarse_inv @ G
    assert abs(lv.w @ x[lv.disc.n_v:]) < 1e-12
    np.testing.assert_allclose(lv.K @ x, G, atol=1e-10 * abs(G).max())


@pytest.mark.parametrize("nu1,nu2,L", [(0, 1, 2), (1, 0, 3), (2, 2, 3), (3, 1, 4), (1, 3, 2)])
def test_divergence_free_after_every_step(nu1, nu2, L):
    """A divergence-free start stays divergence-free after every smoothing step
    and every cycle, for any numbers of pre/post steps and levels."""
    d, N, k = 2, 16, 2
    h = Hierarchy(d, N, k, L, 1.0, 10.0)
    disc = h.finest.disc
    F = load_vector(disc, forcing(d, 1.0, 10.0))
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 11),
                             workloads.random_coefficients(disc.n_q, 12))
    scale = l2_norm_velocity(disc, U)
    assert div_norm(disc, U) < 1e-12 * scale
    et = eta_levels(h, None)
    for _ in range(2):
        U = smooth(h.finest, U, F, et[-1])
        assert div_norm(disc, U) < 1e-12 * scale
    for _ in range(3):
        U = mgv(h, L - 1, U, F, nu1, nu2, et)
        assert div_norm(disc, U) < 1e-12 * scale


def test_divergence_free_3d():
    d, N, k, L = 3, 4, 1, 2
    h = Hierarchy(d, N, k, L, 1.0, 1.0)
    disc = h.finest.disc
    F = load_vector(disc, forcing(d, 1.0, 1.0))
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 1),
                             workloads.random_coefficients(disc.n_q, 2))
    scale = l2_norm_velocity(disc, U)
    U = vcycles(h, U, F, 2, 1, 2)
    assert div_norm(disc, U) < 1e-12 * scale


def _rate(h, F, seed, m=6):
    disc = h.finest.disc
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, seed),
                             workloads.random_coefficients(disc.n_q, seed + 1))
    r0 = residual_norm(h, U, F)
    U = vcycles(h, U, F, m)
    return (residual_norm(h, U, F) / r0) ** (1.0 / m)


@pytest.mark.parametrize("sigma", [1.0, 1e3])
def test_convergence_factor_does_not_grow_with_h(sigma):
    """Coarsest grid fixed at 4x4; the V(2,2) factor stays bounded away from 1
    and does not grow from 16x16 to 64x64 (k=2)."""
    rates = []
    for N, L in ((16, 3), (32, 4), (64, 5)):
        h = Hierarchy(2, N, 2, L, 1.0, sigma)
        F = load_vector(h.finest.disc, forcing(2, 1.0, sigma))
        rates.append(_rate(h, F, 21))
    assert max(rates) < 0.45, rates
    assert rates[-1] <= rates[0] + 0.05, rates


def test_oseen_converges():
    c = workloads.rotation_speed(0.1, 32, 0.5)
    adv = rotation_field(c)
    h = Hierarchy(2, 32, 2, 4, 0.1, 1.0, adv)
    F = load_vector(h.finest.disc, forcing(2, 0.1, 1.0, adv))
    U, hist = solve(h, F, tol=1e-8, max_cycles=100)
    assert hist[-1] <= 1e-8 * np.linalg.norm(F)
    assert div_norm(h.finest.disc, U) < 1e-12 * l2_norm_velocity(h.finest.disc, U)


def test_per_level_smoothing_steps():
    """Per-level step counts: a constant list reproduces the scalar counts, a
    level with zero steps is skipped, and mixed counts keep the velocity
    divergence-free (every correction is a scalar times a divergence-free
    field, whatever the number of steps on each level)."""
    h = Hierarchy(2, 8, 1, 3, 1.0, 1.0)
    F = load_vector(h.finest.disc, forcing(2, 1.0, 1.0))
    U0 = np.zeros_like(F)
    a = vcycles(h, U0, F, 2, 2, 2)
    b = vcycles(h, U0, F, 2, [2, 2], [2, 2])
    np.testing.assert_array_equal(a, b)
    c = vcycles(h, U0, F, 2, [3, 1], [1, 4])
    assert not np.allclose(a, c)
    assert div_norm(h.finest.disc, c) < 1e-12 * l2_norm_velocity(h.finest.disc, c)


def test_3d_asymptotic_factor_two_grids():
    """3D k=1, coarsest grid 4^3: the oracle's asymptotic V(2,2) factor (F = 0,
    random divergence-free start, geometric mean over cycles 21..40) on 8^3
    (2 grids) and 16^3 (3 grids) stays below 0.9 and rises by less than 0.1
    (the GPU test extends this to 32^3 with the argued bound on increments)."""
    f = []
    for N, L in ((8, 2), (16, 3)):
        h = Hierarchy(3, N, 1, L, 1.0, 1.0)
        disc = h.finest.disc
        U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 31),
                                 workloads.random_coefficients(disc.n_q, 32))
        F = np.zeros_like(U)
        r = []
        for _ in range(40):
            U = vcycles(h, U, F, 1)
            r.append(residual_norm(h, U, F))
        f.append((r[-1] / r[-21]) ** (1 / 20))
    assert max(f) < 0.9 and f[1] - f[0] < 0.1, f
