"""Pins of the oracle's assembly: structure, exact integrals and the
discretization error rate of a manufactured solution."""
import numpy as np
import pytest

from oracle.spaces import Discretization
from oracle.assemble import assemble, load_vector, pressure_integrals, rotation_field
from oracle.manufactured import forcing, velocity, pressure
from oracle.diagnostics import direct_solve, l2_error_velocity, div_norm
from oracle.bspline import open_knots, basis
from oracle.refine import greville


def test_structure():
    for d, N, k in [(2, 6, 1), (2, 6, 2), (3, 3, 1)]:
        disc = Discretization(d, N, k)
        m = assemble(disc, 0.3, 2.0)
        A, B = m["A"], m["B"]
        assert abs(B @ np.ones(disc.n_q)).max() < 1e-14  # integral of div v over Omega is 0
        assert abs(A - A.T).max() < 1e-13
        assert np.linalg.eigvalsh(A.toarray()).min() > 0
        w = pressure_integrals(disc)
        np.testing.assert_allclose(w.sum(), 1.0, atol=1e-14)


def test_mass_block_integrates_known_function():
    """sigma-only form on u_x = g(x) h(y) with g = x(1-x) (zero at x=0,1) and
    h = y: integral of g^2 h^2 = 1/30 * 1/3."""
    disc = Discretization(2, 4, 1)
    m = assemble(disc, 0.0, 1.0)
    blk = disc.vel[0]
    coef = []
    for j, f in enumerate((lambda t: t * (1 - t), lambda t: t)):
        q = blk.degrees[j]
        kn = open_knots(disc.N, q)
        xg = greville(kn, q)
        c = np.linalg.solve(basis(kn, q, xg), f(xg))
        coef.append(c[blk.lo[j]:blk.hi[j]])
    u = np.kron(coef[1], coef[0])
    Ax = m["A"][:blk.size, :blk.size]
    np.testing.assert_allclose(u @ (Ax @ u), (1 / 30) * (1 / 3), rtol=1e-12)


@pytest.mark.parametrize("d,k,Ns", [(2, 1, (8, 16, 32)), (2, 2, (8, 16, 32)), (3, 1, (4, 8))])
def test_velocity_error_rate(d, k, Ns):
    errs = []
    for N in Ns:
        disc = Discretization(d, N, k)
        m = assemble(disc, 1.0, 1.0)
        F = load_vector(disc, forcing(d, 1.0, 1.0))
        U = direct_solve(disc, m["K"], F)
        errs.append(l2_error_velocity(disc, U, lambda X: velocity(d, X)))
        assert div_norm(disc, U) < 1e-10  # the lemma: b(u,q)=0 for all q gives div u = 0
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 1 - 0.2, rates


def test_oseen_rotation_manufactured():
    d, k, N = 2, 2, 16
    rates = []
    prev = None
    for N in (8, 16, 32):
        disc = Discretization(d, N, k)
        adv = rotation_field(3.0)
        m = assemble(disc, 0.5, 1.0, adv)
        F = load_vector(disc, forcing(d, 0.5, 1.0, adv))
        U = direct_solve(disc, m["K"], F)
        e = l2_error_velocity(disc, U, lambda X: velocity(d, X))
        if prev is not None:
            rates.append(np.log2(prev / e))
        prev = e
    assert rates[-1] > k + 1 - 0.2, rates
