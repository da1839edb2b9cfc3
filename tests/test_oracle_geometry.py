"""Pins of the oracle's mapped geometries and of the assembly on them
(equations physical_2D and physical_3D; the quarter annulus and hollow
cylinder section of the numerical results).

* The Bezier arc is the unit quarter circle; J and its derivatives equal
  finite differences of the map.
* The identity map reproduces the unit-square / unit-cube assembly.
* The Piola identity: the physical divergence of a pushed-forward velocity
  basis function is its parametric divergence over det J.
* The whole operator on the annulus and on the cylinder section equals an
  independent assembly in cylindrical coordinates (r, theta, z): velocity
  components from the orthogonal frame, the gradient with its Christoffel
  terms, div in polar form, boundary faces with arc-length measure; theta'
  and theta'' are taken by finite differences of atan2 of the map.
* A divergence-free start (curl of potentials) has B^T u = 0.
* The divergence norm on the mapped domain equals the unit-domain norm for
  the identity map and, on the annulus, the quadrature of the physical
  divergence (traces of the physical gradients) against det J.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle.spaces import Discretization
from oracle.assemble import assemble, quadrature, tensor_eval, tensor_points, tensor_weights
from oracle.complex import random_divfree_start
from oracle.geometry import IdentityMap, QuarterAnnulus, assemble_mapped, physical_basis, div_norm_mapped
from oracle.diagnostics import div_norm


def test_arc_and_jacobian():
    t = np.linspace(0.0, 1.0, 41)
    c, _, _ = QuarterAnnulus.arc(t)
    np.testing.assert_allclose(np.linalg.norm(c, axis=1), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(c[0], [1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(c[-1], [0.0, 1.0], atol=1e-15)
    assert np.all(np.diff(np.arctan2(c[:, 1], c[:, 0])) > 0)
    for d in (2, 3):
        g = QuarterAnnulus(d)
        rng = np.random.default_rng(1)
        Xi = 0.1 + 0.8 * rng.random((20, d))
        x, J, dJ = g.geometry(Xi)
        eps = 1e-4
        for m in range(d):
            e = np.zeros(d)
            e[m] = eps
            xs = [g.geometry(Xi + s * e) for s in (-2, -1, 1, 2)]
            fd_x = (xs[0][0] - 8 * xs[1][0] + 8 * xs[2][0] - xs[3][0]) / (12 * eps)
            fd_J = (xs[0][1] - 8 * xs[1][1] + 8 * xs[2][1] - xs[3][1]) / (12 * eps)
            np.testing.assert_allclose(J[:, :, m], fd_x, rtol=0, atol=1e-10)
            np.testing.assert_allclose(dJ[:, m], fd_J, rtol=0, atol=1e-9)


@pytest.mark.parametrize("d,N,k", [(2, 4, 1), (2, 3, 2), (3, 2, 1)])
def test_identity_map_is_unit_domain(d, N, k):
    disc = Discretization(d, N, k)
    got = assemble_mapped(disc, IdentityMap(d), 0.7, 3.0)["K"]
    want = assemble(disc, 0.7, 3.0)["K"]
    assert abs(got - want).max() <= 1e-13 * abs(want).max()


@pytest.mark.parametrize("d", [2, 3])
def test_piola_divergence(d):
    disc = Discretization(d, 3, 2)
    g = QuarterAnnulus(d)
    pts, _ = quadrature(disc)
    for c in range(d):
        _, T, det = physical_basis(disc, g, c, pts)
        div = sum(T[i][i] for i in range(d))
        ref = sp.diags(1.0 / det) @ tensor_eval(disc, disc.vel[c], pts, deriv_dir=c)
        assert abs(div - ref).max() <= 1e-10 * abs(ref).max()


def _theta_derivs(t):
    """theta(t) = atan2 of the arc and its first two derivatives (finite
    differences of fourth order)."""
    def th(s):
        c, _, _ = QuarterAnnulus.arc(s)
        return np.arctan2(c[:, 1], c[:, 0])
    h = 1e-3
    f = [th(t + j * h) for j in (-2, -1, 0, 1, 2)]
    d1 = (f[0] - 8 * f[1] + 8 * f[3] - f[4]) / (12 * h)
    d2 = (-f[0] + 16 * f[1] - 30 * f[2] + 16 * f[3] - f[4]) / (12 * h * h)
    return th(t), d1, d2


def _cylindrical_fields(disc, g, pts):
    """Per velocity component c: the function S_c and unit direction index
    of the physical field (v = S_c N e_dir), and the cylindrical gradient
    G[a][b] (component a in (e_r, e_theta, e_z), derivative along b), all as
    sparse matrices over the tensor grid pts; with the area factor."""
    d = disc.d
    Xi = tensor_points(pts)
    dr, D = g.r_out - g.r_in, (g.depth if d == 3 else 1.0)
    r = g.r_in + dr * Xi[:, 0]
    _, tp, tpp = _theta_derivs(Xi[:, 1])
    vol = dr * r * tp * D
    out = []
    for c, blk in enumerate(disc.vel):
        N = tensor_eval(disc, blk, pts)
        dN = [tensor_eval(disc, blk, pts, deriv_dir=q) for q in range(d)]
        # v = S N e_c with S = dr / vol, r tp / vol, D / vol (frame r, theta, z)
        if c == 0:
            S, dS = 1.0 / (r * tp * D), [-dr / (r ** 2 * tp * D), -tpp / (r * tp ** 2 * D)]
        elif c == 1:
            S, dS = 1.0 / (dr * D) + 0 * r, [0 * r, 0 * r]
        else:
            S, dS = 1.0 / (dr * r * tp), [-1.0 / (r ** 2 * tp), -tpp / (dr * r * tp ** 2)]
        if d == 3:
            dS.append(0 * r)
        # d/dxi_q of the nonzero component f = S N
        dF = [sp.diags(dS[q]) @ N + sp.diags(S) @ dN[q] for q in range(d)]
        F = sp.diags(S) @ N
        Z = sp.csr_matrix(F.shape)
        comp = [Z] * d
        comp[c] = F
        dcomp = [[Z] * d for _ in range(d)]   # dcomp[a][q]
        for q in range(d):
            dcomp[c][q] = dF[q]
        scale = [1.0 / dr + 0 * r, 1.0 / tp, 1.0 / D + 0 * r]   # d/dr, d/dtheta, d/dz from d/dxi
        G = [[None] * d for _ in range(d)]
        G[0][0] = sp.diags(scale[0]) @ dcomp[0][0]
        G[0][1] = sp.diags(1.0 / r) @ (sp.diags(scale[1]) @ dcomp[0][1] - comp[1])
        G[1][0] = sp.diags(scale[0]) @ dcomp[1][0]
        G[1][1] = sp.diags(1.0 / r) @ (sp.diags(scale[1]) @ dcomp[1][1] + comp[0])
        if d == 3:
            G[0][2] = sp.diags(scale[2]) @ dcomp[0][2]
            G[1][2] = sp.diags(scale[2]) @ dcomp[1][2]
            G[2][0] = sp.diags(scale[0]) @ dcomp[2][0]
            G[2][1] = sp.diags(1.0 / r) @ sp.diags(scale[1]) @ dcomp[2][1]
            G[2][2] = sp.diags(scale[2]) @ dcomp[2][2]
        div = sum(G[a][a] for a in range(d))
        out.append((comp, G, div))
    return out, vol, r, tp


def _cylindrical_assembly(disc, g, nu, sigma):
    d, k = disc.d, disc.k
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    fields, vol, _, _ = _cylindrical_fields(disc, g, pts)
    Wv = sp.diags(w * vol)
    A = [[None] * d for _ in range(d)]
    for c in range(d):
        for c2 in range(d):
            v, Gv, _ = fields[c]
            u, Gu, _ = fields[c2]
            A[c][c2] = sigma * sum(v[a].T @ Wv @ u[a] for a in range(d)) + \
                nu * sum(Gv[a][b].T @ Wv @ Gu[a][b] for a in range(d) for b in range(d))
    dr, D = g.r_out - g.r_in, (g.depth if d == 3 else 1.0)
    for e in range(d):
        for side, sgn in ((0.0, -1.0), (1.0, 1.0)):
            fp, fw = list(pts), list(wts)
            fp[e], fw[e] = np.array([side]), np.array([1.0])
            ff, _, r, tp = _cylindrical_fields(disc, g, fp)
            # arc length per unit parameter of the face and the normal element size
            if e == 0:
                ds, h = r * tp * D, dr / disc.N + 0 * r
            elif e == 1:
                ds, h = dr * D + 0 * r, r * tp / disc.N
            else:
                ds, h = dr * r * tp, D / disc.N + 0 * r
            ws = tensor_weights(fw) * ds
            for c in range(d):
                for c2 in range(d):
                    v, Gv, _ = ff[c]
                    u, Gu, _ = ff[c2]
                    for a in range(d):
                        dnu = sgn * Gu[a][e]
                        dnv = sgn * Gv[a][e]
                        A[c][c2] = A[c][c2] - nu * (v[a].T @ sp.diags(ws) @ dnu) - nu * (dnv.T @ sp.diags(ws) @ u[a]) \
                            + 4.0 * k * nu * (v[a].T @ sp.diags(ws / h) @ u[a])
    Phi_q = tensor_eval(disc, disc.pre, pts)
    B = sp.vstack([fields[c][2].T @ sp.diags(w) @ Phi_q for c in range(d)], format="csr")
    A = sp.csr_matrix(sp.bmat(A))
    return sp.bmat([[A, -B], [B.T, None]], format="csr")


@pytest.mark.parametrize("d,N,k", [(2, 3, 1), (2, 2, 2), (3, 2, 1)])
def test_annulus_against_cylindrical_coordinates(d, N, k):
    disc = Discretization(d, N, k)
    g = QuarterAnnulus(d)
    got = assemble_mapped(disc, g, 0.6, 40.0)["K"]
    want = _cylindrical_assembly(disc, g, 0.6, 40.0)
    err = abs(got - want).max() / abs(want).max()
    assert err <= 1e-9, err
    # the cross-component blocks are present (the map couples components)
    nv0 = disc.offsets[1]
    assert abs(got[:nv0, nv0:disc.offsets[2]]).max() > 1e-3 * abs(got).max()


@pytest.mark.parametrize("d,N,k", [(2, 4, 1), (2, 4, 2), (3, 3, 1)])
def test_divergence_free_start_on_annulus(d, N, k):
    disc = Discretization(d, N, k)
    B = assemble_mapped(disc, QuarterAnnulus(d), 1.0, 1.0)["B"]
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 5),
                             workloads.random_coefficients(disc.n_q, 6))
    u = U[:disc.n_v]
    assert np.abs(B.T @ u).max() <= 1e-13 * np.abs(B).max() * np.abs(u).max()


@pytest.mark.parametrize("d,N,k", [(2, 4, 1), (2, 3, 2), (3, 2, 1)])
def test_div_norm_mapped(d, N, k):
    disc = Discretization(d, N, k)
    U = workloads.random_coefficients(disc.n, 9)
    assert abs(div_norm_mapped(disc, IdentityMap(d), U) - div_norm(disc, U)) <= 1e-14 * div_norm(disc, U)
    g = QuarterAnnulus(d)
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    div = 0.0
    for c in range(d):
        _, T, det = physical_basis(disc, g, c, pts)
        div = div + sum(T[i][i] for i in range(d)) @ U[disc.offsets[c]:disc.offsets[c + 1]]
    want = np.sqrt(np.sum(w * det * div * div))
    assert abs(div_norm_mapped(disc, g, U) - want) <= 1e-10 * want
