"""Generalized Oseen problems as the paper poses them (advection equal to the
manufactured velocity, 2D and 3D) and the 3D rotation, through the C-ABI
against the oracle: V-cycles with the additive and the multiplicative
smoother (velocity 1e-10 relative L2), solves (equal cycle counts), the FP32
refinement (1e-8), and the paper's protocol for the Re = 1 rows of its
Table 6 (2D, multiplicative, within two cycles)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle.multigrid import Hierarchy, vcycles, solve, residual_norm
from oracle.assemble import load_vector, rotation_field
from oracle.manufactured import forcing, manufactured_advection
from oracle.complex import random_divfree_start
from oracle.diagnostics import div_norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cycle_tables.json")))
UMAX = {2: np.pi, 3: np.pi * np.sqrt(2.0)}   # max |u| of the manufactured velocity


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def field(d, c, kind):
    return {1: rotation_field(c), 2: manufactured_advection(d, c)}[kind]


def make(d, N, k, L, nu, sigma, c, kind, **opt):
    from paper_1705_09282_amd.dfmg import Solver
    print(f"\n[case] oseen d={d} N={N} k={k} L={L} nu={nu} sigma={sigma} c={c} kind={kind} opt={opt}", flush=True)
    s = Solver(d, N, L, k, nu=nu, sigma=sigma, c=c, adv_kind=kind, **opt).bind()
    adv = field(d, c, kind)
    h = Hierarchy(d, N, k, L, nu, sigma, adv)
    F = load_vector(h.finest.disc, forcing(d, nu, sigma, adv))
    return s, h, F


CASES = [(2, 16, 1, 3, 1.0, 1.0, 20.0, 2), (2, 16, 2, 3, 0.1, 1.0, 0.5, 2), (3, 8, 1, 3, 1.0, 10.0, 5.0, 2),
         (3, 8, 1, 3, 1.0, 1.0, 8.0, 1)]


@pytest.mark.parametrize("d,N,k,L,nu,sigma,c,kind", CASES)
@pytest.mark.parametrize("mult", [0, 1])
def test_oseen_cycles_match_oracle(d, N, k, L, nu, sigma, c, kind, mult):
    s, h, F = make(d, N, k, L, nu, sigma, c, kind, multiplicative=mult, nu1=1, nu2=2)
    disc = h.finest.disc
    U0 = random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, 51),
                              workloads.random_coefficients(disc.n_q, 52))
    Ud = dev(U0)
    s.vcycle(dev(F), Ud, 3)
    Uo = vcycles(h, U0, F, 3, 1, 2, smoother="multiplicative" if mult else "additive")
    got = Ud.cpu().numpy()
    nv = disc.n_v
    assert rel_l2(got[:nv], Uo[:nv]) < 1e-10
    assert div_norm(disc, got) < 1e-10 * max(1.0, np.linalg.norm(got[:nv]))
    s.close()


@pytest.mark.parametrize("d,N,k,L,nu,sigma,c,kind", CASES[:3])
def test_oseen_solve_matches_oracle(d, N, k, L, nu, sigma, c, kind):
    s, h, F = make(d, N, k, L, nu, sigma, c, kind, max_cycles=300)
    Ud = dev(np.zeros_like(F))
    st = s.solve(dev(F), Ud, tol=1e-8)
    Uo, hist = solve(h, F, tol=1e-8, max_cycles=300)
    nv = h.finest.disc.n_v
    print(f"[oseen] cycles gpu {st['cycles']} oracle {len(hist) - 1}", flush=True)
    assert st["converged"] and st["cycles"] == len(hist) - 1
    assert rel_l2(Ud.cpu().numpy()[:nv], Uo[:nv]) < 1e-10
    assert s.div_norm(Ud) < 1e-10
    s.close()


def test_oseen_fp32_refinement_matches_oracle():
    d, N, k, L, nu, sigma, c = 2, 32, 2, 4, 1.0, 1.0, 2.0
    s, h, F = make(d, N, k, L, nu, sigma, c, 2, precision=1)
    Ud = dev(np.zeros_like(F))
    st = s.solve(dev(F), Ud, tol=1e-10)
    Uo, _ = solve(h, F, tol=1e-12, max_cycles=400)
    nv = h.finest.disc.n_v
    err = rel_l2(Ud.cpu().numpy()[:nv], Uo[:nv])
    print(f"[oseen fp32] steps {st['cycles']} vel rel err {err:.2e} div {s.div_norm(Ud):.1e}", flush=True)
    assert st["converged"] and err < 1e-8 and s.div_norm(Ud) < 1e-10
    s.close()


def _divfree(disc, seed=0):
    return random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, seed),
                                workloads.random_coefficients(disc.n_q, seed + 1))


@pytest.mark.parametrize("Da,key", [(1.0, "Re1Da1"), (1000.0, "Re1Da1000")])
def test_table6_re1_rows(Da, key):
    """The paper's 2D Oseen protocol (multiplicative V(1,2), advection the
    manufactured velocity scaled to max |a| / nu = Re = 1, sigma / nu = Da,
    nu = 1, coarsest grid one element, residual reduced by 1e6 from a random
    divergence-free start): within two cycles of Table 6 for n_l = 2..8."""
    from paper_1705_09282_amd.dfmg import Solver
    from oracle.spaces import Discretization
    paper = GOLD["table6_oseen_2d"][key]
    counts = []
    for nl in range(2, 9):
        N, L = 2 ** nl, nl + 1
        print(f"\n[case] table6 n_l={nl} {key}", flush=True)
        s = Solver(2, N, L, 1, nu=1.0, sigma=Da, c=1.0 / UMAX[2], adv_kind=2, multiplicative=1, nu1=1, nu2=2).bind()
        U, F = dev(_divfree(Discretization(2, N, 1))), dev(s.manufactured_rhs())
        r0 = s.residual_norm(F, U)
        c = 0
        while s.residual_norm(F, U) > 1e-6 * r0 and c < 40:
            s.vcycle(F, U, 1)
            c += 1
        counts.append(c)
        s.close()
    print(f"[table6] {key} gpu n_l=2..8: {counts}; paper {paper[1:8]}", flush=True)
    for nl, c in zip(range(2, 9), counts):
        assert abs(c - paper[nl - 1]) <= 2, (nl, c, paper[nl - 1])
