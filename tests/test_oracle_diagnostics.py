"""Pins of the oracle's diagnostics against closed forms.

u = (x(1-x) y^m, 0) lies in the velocity space for every k >= 1: x(1-x) is a
polynomial of degree 2 <= k+1 that vanishes at x = 0 and x = 1, so its
B-spline coefficients on the two end functions (the only ones non-zero on
those faces) are zero, and y^m (m <= 1 <= k) is a spline of degree k.  Its
coefficients are the polar forms (blossoms) of the polynomials at the knots
(Marsden's identity): for degree q and function i, the symmetric multi-affine
form of the polynomial evaluated at t_{i+1}, ..., t_{i+q}.  That gives
exact coefficients without evaluating any basis function, and
||div u||_L2 = ||(1 - 2x) y^m|| = 1/sqrt(3 (2m + 1)),
||u||_L2 = 1/sqrt(30 (2m + 1)) on the unit square (factors 1/3 per extra
direction of y^m z^m in 3D)."""
import itertools
import math

import numpy as np
import pytest

from oracle.spaces import Discretization
from oracle.bspline import open_knots
from oracle.diagnostics import div_norm, l2_norm_velocity
from oracle.refine import prolongation, potential_prolongation
from oracle.complex import curl


def _blossom_coeffs(knots, q, poly):
    """Coefficients of the polynomial sum_j poly[j] x^j (degree <= q) in the
    degree-q B-spline basis on `knots`: c_i = polar form at t_{i+1..i+q}."""
    n = len(knots) - q - 1
    out = np.zeros(n)
    for i in range(n):
        t = knots[i + 1:i + q + 1]
        c = 0.0
        for j, a in enumerate(poly):
            if a == 0.0:
                continue
            # elementary symmetric polynomial e_j(t) / binom(q, j)
            e = sum(math.prod(s) for s in itertools.combinations(t, j)) if j else 1.0
            c += a * e / math.comb(q, j)
        out[i] = c
    return out


def _field(d, N, k, comp, m):
    """U of u with component `comp` equal to x_c (1 - x_c) * prod_{j != c} x_j^m,
    the others zero, and zero pressure."""
    disc = Discretization(d, N, k)
    U = np.zeros(disc.n)
    blk = disc.vel[comp]
    per_dir = []
    for j in range(d):
        q = blk.degrees[j]
        kn = open_knots(N, q)
        poly = [0.0, 1.0, -1.0] if j == comp else ([0.0] * m + [1.0])
        c = _blossom_coeffs(kn, q, poly)
        if j == comp:
            assert abs(c[0]) < 1e-15 and abs(c[-1]) < 1e-15   # the removed end functions carry nothing
        per_dir.append(c[blk.lo[j]:blk.hi[j]])
    coef = per_dir[0]
    for j in range(1, d):
        coef = np.kron(per_dir[j], coef)     # x fastest
    U[disc.offsets[comp]:disc.offsets[comp + 1]] = coef
    return disc, U


@pytest.mark.parametrize("d,N,k,comp,m", [(2, 4, 1, 0, 0), (2, 8, 1, 0, 1), (2, 8, 2, 1, 1), (2, 5, 2, 0, 1),
                                          (3, 4, 1, 0, 1), (3, 3, 1, 2, 1), (3, 2, 2, 1, 0)])
def test_div_norm_and_l2_norm_closed_form(d, N, k, comp, m):
    disc, U = _field(d, N, k, comp, m)
    other = 1.0 / (2 * m + 1)
    exact_div = math.sqrt(other ** (d - 1) / 3.0)
    exact_l2 = math.sqrt(other ** (d - 1) / 30.0)
    assert abs(div_norm(disc, U) - exact_div) <= 1e-12 * exact_div
    assert abs(l2_norm_velocity(disc, U) - exact_l2) <= 1e-12 * exact_l2


@pytest.mark.parametrize("d,Nc,k", [(2, 4, 1), (2, 4, 2), (3, 2, 1)])
def test_potential_prolongation_commutes_with_curl(d, Nc, k):
    """Refinement commutes with the complex (nested complexes): the curl of a
    refined potential is the refined curl, C_f P^psi psi = P^v C_c psi."""
    dc, df = Discretization(d, Nc, k), Discretization(d, 2 * Nc, k)
    Ps = potential_prolongation(dc, df)
    Pv = prolongation(dc, df)[:df.n_v, :dc.n_v]
    psi = np.random.default_rng(7).uniform(-1, 1, dc.n_psi)
    lhs = curl(df, Ps @ psi)
    rhs = Pv @ curl(dc, psi)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-11 * abs(rhs).max())


def _tensor_coeffs(disc, blk, polys):
    """Blossom coefficients of prod_j polys[j](x_j) in block `blk`."""
    per_dir = []
    for j, poly in enumerate(polys):
        q = blk.degrees[j]
        c = _blossom_coeffs(open_knots(disc.N, q), q, poly)
        per_dir.append(c[blk.lo[j]:blk.hi[j]])
    coef = per_dir[0]
    for j in range(1, len(polys)):
        coef = np.kron(per_dir[j], coef)
    return coef


@pytest.mark.parametrize("d,N,k", [(2, 4, 1), (2, 6, 2), (3, 3, 1), (3, 2, 2)])
def test_curl_closed_form(d, N, k):
    """psi = x(1-x) y(1-y) (2D streamfunction; in 3D the z-component of the
    vector potential, constant in z) has curl (d_y psi, -d_x psi[, 0]) =
    (x(1-x)(1-2y), -(1-2x)y(1-y)[, 0]) (the 2D sign u = (d_y psi, -d_x psi)).
    Both sides are exact spline coefficients from polar forms."""
    disc = Discretization(d, N, k)
    xx, one, lin = [0.0, 1.0, -1.0], [1.0], [1.0, -2.0]
    pb = disc.pot[0] if d == 2 else disc.pot[2]
    psi = np.zeros(disc.n_psi)
    polys = [xx, xx] + ([one] if d == 3 else [])
    off = 0 if d == 2 else disc.pot_offsets[2]
    psi[off:off + pb.size] = _tensor_coeffs(disc, pb, polys)
    want = np.zeros(disc.n_v)
    ux = [xx, lin] + ([one] if d == 3 else [])
    uy = [lin, xx] + ([one] if d == 3 else [])
    want[disc.offsets[0]:disc.offsets[1]] = _tensor_coeffs(disc, disc.vel[0], ux)
    want[disc.offsets[1]:disc.offsets[2]] = -_tensor_coeffs(disc, disc.vel[1], uy)
    got = curl(disc, psi)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
