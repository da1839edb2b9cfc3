"""Pins of the additive-Schwarz damping reading (equation ASM's factor eta).

The paper runs the additive smoother with eta = 0.5 (numerical-results
section) and calls eta a suitably chosen factor in (0, 1).  Read literally
(plain sum of the local corrections, zero-mean local pressure), S^-1 K has
eigenvalues up to lambda_max = 4.9 (2D, k = 1), 9.0 (2D, k = 2), 24 (3D,
k = 1), 80 (3D, k = 2), so the damped step amplifies those modes unless
eta lambda_max < 2.  The oracle's fixed damping eta0 is the value of a sweep
with the fewest V(2,2) cycles among those with eta lambda_max <= 1.85.  These
tests pin that reading against the paper's protocol (V(1,2), a single
coarsest element, a random divergence-free start, residual reduced by 1e6)
and the paper's Table 2."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads
from oracle.multigrid import (Hierarchy, residual_norm, vcycles, solve, schwarz_correction, default_eta,
                              SWEEP_ETA, ETA_MARGIN)
from oracle.assemble import load_vector
from oracle.manufactured import forcing
from oracle.complex import random_divfree_start

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cycle_tables.json")))


def _lmax(lv):
    """Largest |eigenvalue| of S^-1 K of a level (ARPACK)."""
    X = sla.LinearOperator((lv.disc.n,) * 2, matvec=lambda v: schwarz_correction(lv, lv.K @ v))
    ev = sla.eigs(X, k=1, which="LM", return_eigenvectors=False, tol=1e-10, maxiter=20000)
    return float(abs(ev[0]))


def _paper_protocol(d, k, nl, sigma, eta, max_cycles, smoother="additive", seed=0):
    """Cycles of V(1,2) from a random divergence-free start until the residual
    drops by 1e6 (numerical-results protocol, single coarsest element);
    returns (cycles, final ratio)."""
    N, L = 2 ** nl, nl + 1
    h = Hierarchy(d, N, k, L, 1.0, sigma)
    disc = h.finest.disc
    F = load_vector(disc, forcing(d, 1.0, sigma))
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, seed),
                             workloads.random_coefficients(disc.n_q, seed + 1))
    r0 = residual_norm(h, U, F)
    c, r = 0, r0
    while r > 1e-6 * r0 and c < max_cycles and r < 1e3 * r0:
        U = vcycles(h, U, F, 1, 1, 2, eta=eta, smoother=smoother)
        c += 1
        r = residual_norm(h, U, F)
    return c, r / r0


def test_paper_eta_half_diverges_and_eta0_converges():
    """2D, k = 1 (the paper's p = 2), 16x16, V(1,2): with eta = 0.5 the
    residual grows, with eta0 it drops by 1e6 within 25 cycles."""
    c, ratio = _paper_protocol(2, 1, 4, 1.0, 0.5, 40)
    assert ratio > 1.0, (c, ratio)
    c, ratio = _paper_protocol(2, 1, 4, 1.0, default_eta(2, 1), 25)
    assert ratio <= 1e-6, (c, ratio)


@pytest.mark.parametrize("d,k,N,L", [(2, 1, 16, 3), (2, 2, 16, 3), (3, 1, 8, 3), (3, 2, 4, 2)])
def test_eta0_is_best_sweep_value_within_margin(d, k, N, L):
    """eta0 lambda_max < 2 on every smoothed level, and among the sweep values
    with eta lambda_max <= 1.85 on the finest level, eta0 needs the fewest
    V(2,2) cycles to 1e-8 from U = 0 (within one cycle); a sweep value past
    the margin exists (eta0 is limited by stability, not by the sweep)."""
    h = Hierarchy(d, N, k, L, 1.0, 1.0)
    eta0 = default_eta(d, k)
    lams = [_lmax(h.levels[l]) for l in range(1, L)]
    for lam in lams:
        assert eta0 * lam < 2.0, (eta0, lams)
    lam = lams[-1]
    allowed = [e for e in SWEEP_ETA[(d, k)] if e * lam <= ETA_MARGIN]
    assert eta0 in allowed
    assert any(e * lam > ETA_MARGIN for e in SWEEP_ETA[(d, k)])
    F = load_vector(h.finest.disc, forcing(d, 1.0, 1.0))
    cycles = {}
    for e in allowed:
        U, hist = solve(h, F, tol=1e-8, eta=e, max_cycles=300)
        assert hist[-1] <= 1e-8 * np.linalg.norm(F), e
        cycles[e] = len(hist) - 1
    assert cycles[eta0] <= min(cycles.values()) + 1, cycles


@pytest.mark.parametrize("sigma,key", [(1.0, "Da1"), (1000.0, "Da1000")])
def test_table2_soft_comparison(sigma, key):
    """Table 2 (additive, p = 2, V(1,2)): the paper needs 14-16 cycles for
    n_l = 3..6 with eta = 0.5.  With eta0 = 0.35 (eta = 0.5 diverges here)
    the oracle needs between 0.75 and 1.4 times the paper's count (13-21)."""
    paper = GOLD["table2_additive_p2_eta_half"][key]
    for nl in (3, 4, 5, 6):
        c, ratio = _paper_protocol(2, 1, nl, sigma, default_eta(2, 1), 60)
        assert ratio <= 1e-6
        assert 0.75 * paper[nl - 1] <= c <= 1.4 * paper[nl - 1], (nl, c, paper[nl - 1])
