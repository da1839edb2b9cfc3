"""Pins of the oracle's subdomains and local solves."""
import json
import os

import numpy as np
import pytest

from oracle.spaces import Discretization
from oracle.assemble import assemble, pressure_integrals
from oracle.patches import build_patches, local_inverses, submatrices

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_dof_tables.json")))


@pytest.mark.parametrize("d,N,k", [(2, 8, 1), (2, 8, 2), (3, 6, 1)])
def test_interior_subdomain_dimensions(d, N, k):
    """dim V_i = 4, dim Q_i = 4 - 1 (zero mean), dim Psi_i = 1 for interior subdomains."""
    g = GOLD["section_subdomains_interior_dims"]
    disc = Discretization(d, N, k)
    P = build_patches(disc)
    sizes = np.diff(P["ptr"])
    for i in range(len(sizes)):
        o, *mi = P["pot"][i]
        pb = disc.pot[o]
        interior = all(pb.lo[j] + k + 1 <= mi[j] < pb.hi[j] - k - 1 for j in range(d))
        if interior:
            assert P["nv"][i] == g["dim_V_i"]
            assert sizes[i] - P["nv"][i] == g["dim_Q_i_before_mean_zero"]
            assert P["npsi"][i] == g["dim_Psi_i"]


@pytest.mark.parametrize("d,N,k", [(2, 8, 1), (2, 8, 2), (3, 4, 1)])
def test_local_exactness_and_cover(d, N, k):
    """Every local complex is exact: div maps V_i onto the zero-mean part of the
    local pressure span, i.e. rank B_i = n_q,i - 1; the subdomains cover all DOFs."""
    disc = Discretization(d, N, k)
    m = assemble(disc, 1.0, 1.0)
    B = m["B"].toarray()
    P = build_patches(disc)
    covered = np.zeros(disc.n, bool)
    for i in range(len(P["ptr"]) - 1):
        I = P["dofs"][P["ptr"][i]:P["ptr"][i + 1]]
        covered[I] = True
        nv = P["nv"][i]
        Bi = B[np.ix_(I[:nv], I[nv:] - disc.n_v)]
        s = np.linalg.svd(Bi, compute_uv=False)
        rank = int((s > 1e-10 * s.max()).sum())
        assert rank == len(I) - nv - 1
    assert covered.all()


@pytest.mark.parametrize("d,N,k", [(2, 12, 1), (2, 12, 2), (3, 6, 1)])
def test_colours_are_dof_disjoint(d, N, k):
    disc = Discretization(d, N, k)
    P = build_patches(disc)
    ncol = len(np.unique(P["color"]))
    assert ncol == (3 if d == 3 else 1) * (k + 1) ** d
    for c in np.unique(P["color"]):
        ids = np.nonzero(P["color"] == c)[0]
        allidx = np.concatenate([P["dofs"][P["ptr"][i]:P["ptr"][i + 1]] for i in ids])
        assert len(np.unique(allidx)) == allidx.size


def test_local_inverse_solves_bordered_problem():
    disc = Discretization(2, 6, 2)
    m = assemble(disc, 1.0, 5.0)
    P = build_patches(disc)
    w = pressure_integrals(disc)
    rng = np.random.default_rng(7)
    for ids, I, M in local_inverses(m["K"], P, w, disc.n_v):
        Ki = submatrices(m["K"], I)
        e = np.where(I >= disc.n_v, w[np.maximum(I - disc.n_v, 0)], 0.0)
        for j in range(len(ids)):
            r = rng.standard_normal(I.shape[1])
            x = M[j] @ r
            assert abs(e[j] @ x) < 1e-12                      # zero-mean local pressure
            res = Ki[j] @ x - r
            lam = (res @ e[j]) / (e[j] @ e[j])                # residual is a multiple of e
            np.testing.assert_allclose(res, lam * e[j], atol=1e-10)
