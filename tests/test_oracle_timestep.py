"""Pins of the oracle's Crank-Nicolson / Adams-Bashforth right-hand side
(equation GS of the section on temporal discretization).

* The convective load N(w)_i = (N_i, (w . grad) w) of w = (x(1-x), 0[, 0])
  (a field of the velocity space) is the velocity mass matrix times the spline
  coefficients of the cubic x(1-x)(1-2x) in the first component: k = 2
  velocities have degree 3 in x, so the cubic is in the space (its end
  coefficients vanish), and the coefficients are its polar forms.
* Likewise w = (0, y(1-y)) gives (0, y(1-y)(1-2y)).
* The part of the right-hand side linear in the velocity is
  F2 - K U + 2 sigma M u (velocity rows), isolated by scaling U (quadratic
  terms scale by 4, linear by 2), with M the velocity mass matrix assembled
  independently (sigma = 1, nu = 0, which drops the Nitsche terms).
* The first step (no u^{n-1}) equals a step with u^{n-1} = u^n, and the
  pressure rows are zero.

Guermond's step (equation GO):

* The advection by a discrete field whose coefficients are the polar forms
  of (x(1-x), 0[, 0]) assembles the same operator as the analytic field.
* Advecting the discrete field u by itself, K(u) U - K(0) U is the
  convective load N(u) of the CN/AB pins on the velocity rows (the
  assembly's advection term and the load's quadrature are separate code).
* The load is F2 - K(a) U + 2 sigma M u on the velocity rows (M assembled
  independently) and zero on the pressure rows.
"""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle.spaces import Discretization
from oracle.assemble import assemble
from oracle.bspline import open_knots
from oracle.complex import random_divfree_start
from oracle.timestep import convective_load, cnab_rhs, field_advection, go_rhs


def _blossom(knots, q, poly):
    n = len(knots) - q - 1
    out = np.zeros(n)
    for i in range(n):
        t = knots[i + 1:i + q + 1]
        out[i] = sum(a * (sum(math.prod(c) for c in itertools.combinations(t, j)) if j else 1.0) / math.comb(q, j)
                     for j, a in enumerate(poly) if a != 0.0)
    return out


def _coeffs(disc, comp, polys):
    blk = disc.vel[comp]
    per = []
    for j, poly in enumerate(polys):
        q = blk.degrees[j]
        per.append(_blossom(open_knots(disc.N, q), q, poly)[blk.lo[j]:blk.hi[j]])
    c = per[0]
    for j in range(1, len(polys)):
        c = np.kron(per[j], c)
    return c


@pytest.mark.parametrize("d,N,comp", [(2, 4, 0), (2, 6, 1), (3, 3, 0)])
def test_convective_load_closed_form(d, N, comp):
    k = 2
    disc = Discretization(d, N, k)
    quad, cubic, one = [0.0, 1.0, -1.0], [0.0, 1.0, -3.0, 2.0], [1.0]
    polys_w = [one] * d
    polys_w[comp] = quad
    polys_g = [one] * d
    polys_g[comp] = cubic
    W = np.zeros(disc.n)
    W[disc.offsets[comp]:disc.offsets[comp + 1]] = _coeffs(disc, comp, polys_w)
    got = convective_load(disc, W)
    M = assemble(disc, 0.0, 1.0)["A"]       # nu = 0, sigma = 1: the velocity mass matrix
    want = np.zeros(disc.n)
    g = np.zeros(disc.n_v)
    g[disc.offsets[comp]:disc.offsets[comp + 1]] = _coeffs(disc, comp, polys_g)
    want[:disc.n_v] = M @ g
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("d,N,k", [(2, 8, 1), (2, 6, 2), (3, 4, 1)])
def test_cnab_linear_part_and_first_step(d, N, k):
    nu, sigma = 0.3, 7.0
    disc = Discretization(d, N, k)
    m = assemble(disc, nu, sigma)
    K = m["K"]
    M = assemble(disc, 0.0, 1.0)["A"]
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 3),
                             workloads.random_coefficients(disc.n_q, 4))
    F2 = workloads.random_coefficients(disc.n, 5)
    F2[disc.n_v:] = 0.0
    zero = np.zeros(disc.n)
    # F2 enters once; the velocity terms split into orders 1 and 2 in U
    r1 = cnab_rhs(disc, K, sigma, zero, U) - 0.0
    r2 = cnab_rhs(disc, K, sigma, zero, 2 * U)
    lin = (4 * r1 - r2) / 2
    want = np.zeros(disc.n)
    want[:disc.n_v] = (-(K @ U) + 2 * sigma * np.concatenate([M @ U[:disc.n_v], np.zeros(disc.n_q)]))[:disc.n_v]
    np.testing.assert_allclose(lin, want, rtol=0, atol=1e-11 * np.abs(want).max())
    a = cnab_rhs(disc, K, sigma, F2, U)
    b = cnab_rhs(disc, K, sigma, F2, U, Uold=U)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(a).max())
    assert np.all(a[disc.n_v:] == 0.0)
    np.testing.assert_allclose(a - cnab_rhs(disc, K, sigma, zero, U), np.concatenate([F2[:disc.n_v], np.zeros(disc.n_q)]),
                               rtol=0, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("d,N,k", [(2, 5, 1), (2, 4, 2), (3, 3, 1)])
def test_field_advection_polynomial(d, N, k):
    c = 1.7
    disc = Discretization(d, N, k)
    W = np.zeros(disc.n_v)
    W[:disc.offsets[1]] = _coeffs(disc, 0, [[0.0, 1.0, -1.0]] + [[1.0]] * (d - 1))

    def analytic(X):
        out = np.zeros_like(X)
        out[:, 0] = c * X[:, 0] * (1.0 - X[:, 0])
        return out
    got = assemble(disc, 0.4, 2.0, advection=field_advection(disc, W, c))["K"]
    want = assemble(disc, 0.4, 2.0, advection=analytic)["K"]
    assert abs(got - want).max() <= 1e-13 * abs(want).max()


@pytest.mark.parametrize("d,N,k", [(2, 6, 1), (2, 5, 2), (3, 3, 2)])
def test_field_advection_is_convection(d, N, k):
    disc = Discretization(d, N, k)
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 11),
                             workloads.random_coefficients(disc.n_q, 12))
    Ka = assemble(disc, 0.5, 3.0, advection=field_advection(disc, U[:disc.n_v]))["K"]
    K0 = assemble(disc, 0.5, 3.0)["K"]
    got = (Ka @ U - K0 @ U)
    want = convective_load(disc, U)
    np.testing.assert_allclose(got[:disc.n_v], want[:disc.n_v], rtol=0, atol=1e-12 * np.abs(want).max())
    assert np.all(got[disc.n_v:] == 0.0)


@pytest.mark.parametrize("d,N,k", [(2, 6, 1), (3, 3, 1)])
def test_go_rhs_linear(d, N, k):
    nu, sigma = 0.2, 5.0
    disc = Discretization(d, N, k)
    U = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 21),
                             workloads.random_coefficients(disc.n_q, 22))
    Uo = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 23),
                              workloads.random_coefficients(disc.n_q, 24))
    a = 1.5 * U[:disc.n_v] - 0.5 * Uo[:disc.n_v]
    K = assemble(disc, nu, sigma, advection=field_advection(disc, a))["K"]
    M = assemble(disc, 0.0, 1.0)["A"]
    F2 = workloads.random_coefficients(disc.n, 25)
    F2[disc.n_v:] = 0.0
    got = go_rhs(disc, K, sigma, F2, U)
    want = np.zeros(disc.n)
    want[:disc.n_v] = F2[:disc.n_v] - (K @ U)[:disc.n_v] + 2 * sigma * (M @ U[:disc.n_v])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
