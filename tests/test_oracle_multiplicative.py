"""Pins of the oracle's multiplicative Schwarz smoother (equation MSM).

* The coupling-free colouring really is coupling-free: two subdomains of one
  colour share no DOF and K has no entry between their DOFs (brute force).
* Hence the colour-at-a-time sweep equals the plainly sequential sweep over
  the subdomains in the same order (up to rounding).
* One sweep is the product formula of equation MSM: the error is multiplied
  by prod_i (I - E_i^T K_i^-1 E_i K) (dense, tiny grid, K_i bordered with the
  zero-mean local pressure).
* Every step keeps a divergence-free velocity divergence-free (subsection on
  preservation of the divergence-free constraint: each update is a local
  solution with zero divergence).
* Cycle counts under the paper's protocol against Table 1: within two cycles
  for p = 2 (k = 1), and no more than the paper's for p = 3 (k = 2).
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle.multigrid import (Hierarchy, coupling_free_colours, smooth_multiplicative,
                              smooth_multiplicative_colours, sweep_order, local_inverse_table, vcycles,
                              residual_norm, solve)
from oracle.assemble import load_vector
from oracle.manufactured import forcing
from oracle.complex import random_divfree_start
from oracle.diagnostics import div_norm, l2_norm_velocity, direct_solve

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cycle_tables.json")))


@pytest.mark.parametrize("d,N,k", [(2, 8, 1), (2, 8, 2), (3, 4, 1)])
def test_colouring_is_coupling_free(d, N, k):
    h = Hierarchy(d, N, k, 2, 1.0, 1.0)
    lv = h.finest
    P = lv.patches
    col = coupling_free_colours(lv.disc, P)
    ncol = len(np.unique(col))
    assert ncol == (k + 2) ** d * (1 if d == 2 else 3)
    K = abs(lv.K.toarray()) > 0
    n = lv.disc.n
    for c in np.unique(col):
        ids = np.nonzero(col == c)[0]
        owner = -np.ones(n, int)
        for i in ids:
            I = P["dofs"][P["ptr"][i]:P["ptr"][i + 1]]
            assert (owner[I] < 0).all()          # DOF-disjoint
            owner[I] = i
        for i in ids:
            I = P["dofs"][P["ptr"][i]:P["ptr"][i + 1]]
            reach = np.nonzero(K[I].any(axis=0))[0]
            others = owner[reach]
            assert ((others < 0) | (others == i)).all()   # no coupling to another subdomain of the colour


@pytest.mark.parametrize("d,N,k", [(2, 8, 1), (2, 8, 2), (3, 4, 1)])
def test_colour_sweep_equals_sequential_sweep(d, N, k):
    h = Hierarchy(d, N, k, 2, 1.0, 3.0)
    lv = h.finest
    F = load_vector(lv.disc, forcing(d, 1.0, 3.0))
    rng = np.random.default_rng(4)
    U = rng.standard_normal(lv.disc.n)
    a = smooth_multiplicative(lv, U, F)
    b = smooth_multiplicative_colours(lv, U, F)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * abs(a).max())


def test_sweep_is_the_product_formula():
    """e_new = prod_i (I - E_i^T M_i E_i K) e_old, the product taken in visiting
    order (last subdomain leftmost), for a random error e_old = U - U*."""
    h = Hierarchy(2, 8, 1, 2, 1.0, 1.0)
    lv = h.finest
    n = lv.disc.n
    K = lv.K.toarray()
    F = load_vector(lv.disc, forcing(2, 1.0, 1.0))
    Ustar = direct_solve(lv.disc, lv.K, F)
    rng = np.random.default_rng(9)
    U = Ustar + rng.standard_normal(n)
    Unew = smooth_multiplicative(lv, U, F)
    tab = local_inverse_table(lv)
    E = np.eye(n)
    for i in sweep_order(lv):
        I, M = tab[int(i)]
        T = np.eye(n)
        T[np.ix_(I, np.arange(n))] -= M @ K[I, :]
        E = T @ E
    np.testing.assert_allclose(Unew - Ustar, E @ (U - Ustar), rtol=0, atol=1e-10 * abs(U - Ustar).max())


@pytest.mark.parametrize("d,N,k,L", [(2, 16, 2, 3), (3, 4, 1, 2)])
def test_divergence_free_after_every_multiplicative_step(d, N, k, L):
    h = Hierarchy(d, N, k, L, 1.0, 10.0)
    disc = h.finest.disc
    F = load_vector(disc, forcing(d, 1.0, 10.0))
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 5),
                             workloads.random_coefficients(disc.n_q, 6))
    scale = l2_norm_velocity(disc, U)
    for _ in range(2):
        U = smooth_multiplicative(h.finest, U, F)
        assert div_norm(disc, U) < 1e-12 * scale
    for nu1, nu2 in ((1, 2), (0, 1), (2, 0)):
        U = vcycles(h, U, F, 1, nu1, nu2, smoother="multiplicative")
        assert div_norm(disc, U) < 1e-12 * scale


def test_multiplicative_solve_reaches_direct_solution():
    h = Hierarchy(2, 16, 2, 3, 1.0, 1.0)
    disc = h.finest.disc
    F = load_vector(disc, forcing(2, 1.0, 1.0))
    U, hist = solve(h, F, tol=1e-13, nu1=1, nu2=2, smoother="multiplicative", max_cycles=60)
    Ud = direct_solve(disc, h.finest.K, F)
    nv = disc.n_v
    assert np.linalg.norm(U[:nv] - Ud[:nv]) <= 1e-10 * np.linalg.norm(Ud[:nv])


def _protocol_cycles(k, nl, sigma):
    N, L = 2 ** nl, nl + 1
    h = Hierarchy(2, N, k, L, 1.0, sigma)
    disc = h.finest.disc
    F = load_vector(disc, forcing(2, 1.0, sigma))
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 0),
                             workloads.random_coefficients(disc.n_q, 1))
    r0 = residual_norm(h, U, F)
    c = 0
    while residual_norm(h, U, F) > 1e-6 * r0 and c < 40:
        U = vcycles(h, U, F, 1, 1, 2, smoother="multiplicative")
        c += 1
    return c


@pytest.mark.parametrize("sigma,key", [(1.0, "Da1"), (1000.0, "Da1000")])
def test_table1_p2_within_two_cycles(sigma, key):
    paper = GOLD["table1_multiplicative"]["p2"][key]
    for nl in (2, 3, 4, 5, 6):
        c = _protocol_cycles(1, nl, sigma)
        assert abs(c - paper[nl - 1]) <= 2, (nl, c, paper[nl - 1])


@pytest.mark.parametrize("sigma,key", [(1.0, "Da1"), (1000.0, "Da1000")])
def test_table1_p3_no_more_than_paper(sigma, key):
    paper = GOLD["table1_multiplicative"]["p3"][key]
    for nl in (3, 4, 5):
        c = _protocol_cycles(2, nl, sigma)
        assert 4 <= c <= paper[nl - 1], (nl, c, paper[nl - 1])
