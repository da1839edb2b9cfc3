"""Guermond's semi-implicit step (equation GO) through the C-ABI against the
oracle: the operator that advects with a discrete velocity field (advection
kind 3) and the step's load vector, for a batch of two fields (2D and 3D) to
1e-12, and three steps of the scheme from a smooth divergence-free start to
1e-8 with ||div u|| at rounding.  The advection field of step n+1 is
3/2 u^n - 1/2 u^{n-1}, and u^0 at the first step."""
import numpy as np
import pytest

import workloads
from oracle.spaces import Discretization
from oracle.assemble import assemble
from oracle.multigrid import Hierarchy, solve
from oracle.complex import random_divfree_start
from oracle.timestep import field_advection, go_rhs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def start(disc, seed):
    return random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, seed),
                                workloads.random_coefficients(disc.n_q, seed + 1))


def smooth_start(disc, amp=1.0):
    """Curl of the streamfunction sampling amp sin^2(pi x) sin^2(pi y) at the
    Greville points: smooth, divergence-free, |u| about amp * pi."""
    from oracle.bspline import open_knots
    from oracle.refine import greville
    from oracle.complex import curl
    pb = disc.pot[0]
    q = pb.degrees[0]
    x = greville(open_knots(disc.N, q), q)[pb.lo[0]:pb.hi[0]]
    s = np.sin(np.pi * x) ** 2
    return np.concatenate([curl(disc, amp * np.kron(s, s)), np.zeros(disc.n_q)])


@pytest.mark.parametrize("d,N,k,L", [(2, 16, 1, 3), (2, 12, 2, 2), (3, 6, 1, 2)])
def test_go_rhs_matches_oracle(d, N, k, L):
    from paper_1705_09282_amd.dfmg import BatchSolver
    nu, sig = 0.3, [5.0, 200.0]
    print(f"\n[case] guermond rhs d={d} N={N} k={k} L={L}", flush=True)
    disc = Discretization(d, N, k)
    n = disc.n
    fields = [start(disc, 31 + 2 * p)[:disc.n_v] for p in range(2)]
    b = BatchSolver(d, N, L, k, [nu] * 2, sig, cs=[1.0, 1.0], adv_kind=3, adv_coeffs=fields,
                    time_stepping=1).bind()
    U = np.concatenate([start(disc, 3 + 2 * p) for p in range(2)])
    F2 = workloads.random_coefficients(2 * n, 17)
    for p in range(2):
        F2[p * n + disc.n_v:(p + 1) * n] = 0.0
    Fout = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    b.go_rhs(dev(F2), dev(U), Fout)
    got = Fout.cpu().numpy()
    for p in range(2):
        K = assemble(disc, nu, sig[p], advection=field_advection(disc, fields[p]))["K"]
        sl = slice(p * n, (p + 1) * n)
        want = go_rhs(disc, K, sig[p], F2[sl], U[sl])
        err = np.max(np.abs(got[sl] - want)) / np.max(np.abs(want))
        print(f"[guermond] problem {p} rel err {err:.1e}", flush=True)
        assert err < 1e-12
    b.close()


def test_guermond_steps_match_oracle():
    from paper_1705_09282_amd.dfmg import Solver
    d, N, k, L, nu, dt = 2, 16, 2, 3, 0.1, 0.01
    sigma = 2.0 / dt
    disc = Discretization(d, N, k)
    nv = disc.n_v
    U0 = smooth_start(disc)      # |u| about pi: u dt / h about 0.5
    F2 = np.zeros(disc.n)
    Uo_prev, Uo = None, U0.copy()
    Ud_prev, Ud = None, dev(U0)
    for step in range(3):
        a_o = Uo[:nv] if Uo_prev is None else 1.5 * Uo[:nv] - 0.5 * Uo_prev[:nv]
        h = Hierarchy(d, N, k, L, nu, sigma, field_advection(disc, a_o))
        F = go_rhs(disc, h.finest.K, sigma, F2, Uo)
        Unew, _ = solve(h, F, tol=1e-13, U0=Uo, max_cycles=400)
        Uo_prev, Uo = Uo, Unew
        # the GPU step: the field from the device iterates, a fresh context
        cur = Ud.cpu().numpy()[:nv]
        a_d = cur if Ud_prev is None else 1.5 * cur - 0.5 * Ud_prev.cpu().numpy()[:nv]
        s = Solver(d, N, L, k, nu=nu, sigma=sigma, c=1.0, adv_kind=3, adv_coeffs=a_d, time_stepping=1).bind()
        Fd = torch.zeros_like(Ud)
        s.go_rhs(dev(F2), Ud, Fd)
        Unext = Ud.clone()
        st = s.solve(Fd, Unext, tol=1e-12)
        Ud_prev, Ud = Ud, Unext
        got = Ud.cpu().numpy()
        err = np.linalg.norm(got[:nv] - Uo[:nv]) / np.linalg.norm(Uo[:nv])
        print(f"[guermond] step {step + 1}: cycles {st['cycles']} vel rel err {err:.2e} div {s.div_norm(Ud):.1e}",
              flush=True)
        assert err < 1e-8 and s.div_norm(Ud) < 1e-10
        s.close()
