"""Pins of the oracle's knot-insertion refinement and Galerkin hierarchy."""
from math import comb

import numpy as np
import pytest

from oracle.bspline import open_knots, basis
from oracle.refine import refinement_matrix, prolongation, galerkin
from oracle.spaces import Discretization
from oracle.assemble import assemble


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_interior_rows_follow_two_scale_relation(q):
    """Uniform B-spline subdivision: an interior coarse function is
    sum_j binom(q+1, j) / 2^q  N~(2x - j)."""
    Nc = 8
    T = refinement_matrix(Nc, q)
    expect = np.array([comb(q + 1, j) for j in range(q + 2)]) / 2 ** q
    for i in range(q + 1, Nc - 1):
        row = T[i]
        nz = np.nonzero(np.abs(row) > 0)[0]
        np.testing.assert_allclose(row[nz], expect, atol=1e-14)
        assert nz[0] == 2 * i - q


@pytest.mark.parametrize("q", [1, 2, 3])
def test_refinement_reproduces_coarse_functions(q):
    Nc = 5
    T = refinement_matrix(Nc, q)
    x = np.random.default_rng(3).uniform(0, 1, 200)
    Bc = basis(open_knots(Nc, q), q, x)
    Bf = basis(open_knots(2 * Nc, q), q, x)
    np.testing.assert_allclose(Bc, Bf @ T.T, atol=1e-14)
    np.testing.assert_allclose(T.sum(axis=0), 1.0, atol=1e-14)  # partition of unity


def test_galerkin_equals_coarse_assembly_with_fine_h():
    """Nested spaces: R K_fine P is the coarse-grid matrix of the same bilinear
    forms, with the Nitsche h of the fine grid."""
    for d, N, k in [(2, 8, 1), (2, 8, 2), (3, 4, 1)]:
        fine, coarse = Discretization(d, N, k), Discretization(d, N // 2, k)
        Kf = assemble(fine, 0.7, 3.0)["K"]
        Kc = assemble(coarse, 0.7, 3.0, h=1.0 / N)["K"]
        G = galerkin(Kf, prolongation(coarse, fine))
        err = abs(G - Kc).max()
        assert err <= 1e-12 * abs(Kc).max(), err


def test_prolongation_commutes_with_divergence():
    """P^v maps coarse velocities to the same functions on the fine grid, so
    B_fine^T P^v = P^q^T ... checked as: divergence-free coarse fields stay
    divergence-free (b(P u, q) = 0 for all fine q when b(u, q) = 0 coarse)."""
    from oracle.complex import curl
    d, N, k = 2, 8, 2
    fine, coarse = Discretization(d, N, k), Discretization(d, N // 2, k)
    P = prolongation(coarse, fine)
    psi = np.random.default_rng(4).uniform(-1, 1, coarse.n_psi)
    u = curl(coarse, psi)
    U = np.concatenate([u, np.zeros(coarse.n_q)])
    Bf = assemble(fine, 1.0, 1.0)["B"]
    uf = (P @ U)[:fine.n_v]
    assert abs(Bf.T @ uf).max() < 1e-13
