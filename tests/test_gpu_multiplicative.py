"""GPU parity of the multiplicative Schwarz smoother (equation MSM) through
the C-ABI against the oracle's sweep in the same (coupling-free colour)
order: single smoothing steps (1e-12), whole V(1,2) cycles from a random
divergence-free start (velocity 1e-10 relative L2, graph on and off), solves
(equal cycle counts, velocity 1e-10, ||div u|| at rounding), the paper's
protocol for its Table 1 (cycle counts equal to the oracle's where it runs,
within two of the paper's beyond), batches, and the benchmark's 256^2
problems against the oracle's FP64 solution."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle.multigrid import (Hierarchy, smooth_multiplicative, vcycles, solve, residual_norm)
from oracle.assemble import load_vector, rotation_field
from oracle.manufactured import forcing
from oracle.complex import random_divfree_start
from oracle.diagnostics import div_norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cycle_tables.json")))


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(d, N, k, L, nu=1.0, sigma=1.0, c=0.0, **opt):
    from paper_1705_09282_amd.dfmg import Solver
    print(f"\n[case] multiplicative d={d} N={N} k={k} L={L} nu={nu} sigma={sigma} c={c} opt={opt}", flush=True)
    s = Solver(d, N, L, k, nu=nu, sigma=sigma, c=c, multiplicative=1, **opt).bind()
    adv = rotation_field(c) if c else None
    h = Hierarchy(d, N, k, L, nu, sigma, adv)
    F = load_vector(h.finest.disc, forcing(d, nu, sigma, adv))
    return s, h, F


def divfree_start(h, seed):
    disc = h.finest.disc
    return random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, seed),
                                workloads.random_coefficients(disc.n_q, seed + 1))


CASES = [(2, 16, 1, 3, 0.0), (2, 16, 2, 3, 0.0), (3, 8, 1, 3, 0.0), (2, 16, 2, 3, 20.0), (2, 12, 2, 3, 0.0),
         (3, 4, 2, 2, 0.0), (3, 2, 1, 2, 0.0)]


@pytest.mark.parametrize("d,N,k,L,c", CASES)
def test_multiplicative_step_matches_oracle(d, N, k, L, c):
    s, h, F = make(d, N, k, L, sigma=3.0, c=c)
    lv = h.finest
    U0 = np.random.default_rng(7).standard_normal(lv.disc.n)
    Ud = dev(U0)
    s.level_smooth(L - 1, dev(F), Ud, 2)
    Uo = smooth_multiplicative(lv, smooth_multiplicative(lv, U0, F), F)
    got = host(Ud)
    assert np.max(np.abs(got - Uo)) <= 1e-12 * np.max(np.abs(Uo))
    # a coarser level (Galerkin operator)
    l = L - 2
    if l >= 1:
        n = h.levels[l].disc.n
        Fc = np.random.default_rng(8).standard_normal(n)
        V0 = np.random.default_rng(9).standard_normal(n)
        Vd = dev(V0)
        s.level_smooth(l, dev(Fc), Vd, 1)
        Vo = smooth_multiplicative(h.levels[l], V0, Fc)
        assert np.max(np.abs(host(Vd) - Vo)) <= 1e-12 * np.max(np.abs(Vo))
    s.close()


@pytest.mark.parametrize("d,N,k,L,c", CASES)
@pytest.mark.parametrize("graph", [1, 0])
def test_multiplicative_cycles_match_oracle(d, N, k, L, c, graph):
    s, h, F = make(d, N, k, L, c=c, nu1=1, nu2=2, use_graph=graph)
    U0 = divfree_start(h, 23)
    Ud = dev(U0)
    s.vcycle(dev(F), Ud, 3)
    Uo = vcycles(h, U0, F, 3, 1, 2, smoother="multiplicative")
    nv = h.finest.disc.n_v
    got = host(Ud)
    assert rel_l2(got[:nv], Uo[:nv]) < 1e-10
    assert div_norm(h.finest.disc, got) < 1e-10 * max(1.0, np.linalg.norm(got[:nv]))
    s.close()


@pytest.mark.parametrize("d,N,k,L,c", CASES[:4] + CASES[5:])
def test_multiplicative_solve_matches_oracle(d, N, k, L, c):
    s, h, F = make(d, N, k, L, c=c, nu1=1, nu2=2)
    Ud = dev(np.zeros_like(F))
    st = s.solve(dev(F), Ud, tol=1e-8)
    Uo, hist = solve(h, F, tol=1e-8, nu1=1, nu2=2, smoother="multiplicative")
    got = host(Ud)
    nv = h.finest.disc.n_v
    print(f"[mult] cycles gpu {st['cycles']} oracle {len(hist) - 1}", flush=True)
    assert st["converged"] and st["cycles"] == len(hist) - 1
    # residual entries cancel from O(||r_0||) terms: rounding is absolute at ~1e-16 ||r_0||
    np.testing.assert_allclose(st["history"], hist, rtol=1e-9, atol=1e-14 * hist[0])
    assert rel_l2(got[:nv], Uo[:nv]) < 1e-10
    assert abs(h.finest.w @ got[nv:]) < 1e-12
    assert s.div_norm(Ud) < 1e-10
    s.close()


def _divfree(disc, seed=0):
    return random_divfree_start(disc, workloads.random_coefficients(disc.n_psi, seed),
                                workloads.random_coefficients(disc.n_q, seed + 1))


def _gpu_protocol(s, U0, F, max_cycles=40):
    """V-cycles until the residual drops by 1e6 (the paper's protocol)."""
    U, Fd = dev(U0), dev(F)
    r0 = s.residual_norm(Fd, U)
    c = 0
    while s.residual_norm(Fd, U) > 1e-6 * r0 and c < max_cycles:
        s.vcycle(Fd, U, 1)
        c += 1
    return c


@pytest.mark.parametrize("sigma,key", [(1.0, "Da1"), (1000.0, "Da1000")])
def test_table1_protocol_on_gpu(sigma, key):
    """V(1,2) from a random divergence-free start, coarsest grid one element,
    residual reduced by 1e6 (the paper's protocol): the GPU's counts equal
    the oracle's for n_l = 2..5 and stay within two of Table 1 (p = 2) up to
    n_l = 9 (512^2; there the load vector is the library's, whose parity
    with the oracle's is tested elsewhere)."""
    from paper_1705_09282_amd.dfmg import Solver
    from oracle.spaces import Discretization
    paper = GOLD["table1_multiplicative"]["p2"][key]
    counts = []
    for nl in range(2, 10):
        N, L = 2 ** nl, nl + 1
        print(f"\n[case] table1 protocol n_l={nl} sigma={sigma}", flush=True)
        s = Solver(2, N, L, 1, sigma=sigma, multiplicative=1, nu1=1, nu2=2).bind()
        disc = Discretization(2, N, 1)
        U0 = _divfree(disc)
        if nl <= 5:
            h = Hierarchy(2, N, 1, L, 1.0, sigma)
            F = load_vector(disc, forcing(2, 1.0, sigma))
        else:
            h, F = None, s.manufactured_rhs()
        c = _gpu_protocol(s, U0, F)
        counts.append(c)
        if h is not None:
            U = U0.copy()
            r0 = residual_norm(h, U, F)
            co = 0
            while residual_norm(h, U, F) > 1e-6 * r0 and co < 40:
                U = vcycles(h, U, F, 1, 1, 2, smoother="multiplicative")
                co += 1
            assert c == co, (nl, c, co)
        s.close()
    print(f"[table1] sigma={sigma} gpu counts n_l=2..9: {counts}; paper {paper[1:9]}", flush=True)
    for nl, c in zip(range(2, 10), counts):
        assert abs(c - paper[nl - 1]) <= 2, (nl, c, paper[nl - 1])


def test_multiplicative_batch_equals_single():
    from paper_1705_09282_amd.dfmg import BatchSolver, Solver
    sig = [0.01, 1.0, 1e4]
    B = BatchSolver(2, 32, 4, 2, [1.0] * 3, sig, multiplicative=1, nu1=1, nu2=2).bind()
    F = torch.tensor(B.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    st = B.solve(F, U, tol=1e-8)
    n = B.n
    for p, sg in enumerate(sig):
        S = Solver(2, 32, 4, 2, sigma=sg, multiplicative=1, nu1=1, nu2=2).bind()
        Fs = torch.tensor(S.manufactured_rhs(), device="cuda")
        Us = torch.zeros_like(Fs)
        ss = S.solve(Fs, Us, tol=1e-8)
        assert ss["cycles"] == st[p]["cycles"]
        assert torch.equal(Us, U[p * n:(p + 1) * n])
        S.close()
    B.close()


def test_multiplicative_full_size_matches_oracle():
    """The benchmark's four 256^2 problems (k=2, 6 grids) with multiplicative
    V(1,2) as one batch: each converges, is divergence-free, and its velocity
    matches the oracle's solution (solved to 1e-12) within 1e-8."""
    from paper_1705_09282_amd.dfmg import BatchSolver
    sig = list(workloads.STOKES2D_SIGMAS)
    B = BatchSolver(2, 256, 6, 2, [1.0] * 4, sig, multiplicative=1, nu1=1, nu2=2).bind()
    F = torch.tensor(B.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    st = B.solve(F, U, tol=1e-8)
    div = B.div_norm(U)
    print(f"[mult256] cycles {[x['cycles'] for x in st]} div {div.tolist()}", flush=True)
    assert all(x["converged"] for x in st) and div.max() < 1e-10
    Uh = U.cpu().numpy()
    n = B.n
    for p in (1, 3):
        cfg = workloads.stokes2d(sig[p])
        print(f"[case] oracle 256^2 sigma={sig[p]}", flush=True)
        h = Hierarchy(2, 256, 2, 6, 1.0, sig[p])
        Fo = load_vector(h.finest.disc, forcing(2, 1.0, sig[p]))
        Uo, _ = solve(h, Fo, tol=1e-12, max_cycles=400)
        nv = h.finest.disc.n_v
        err = rel_l2(Uh[p * n:p * n + nv], Uo[:nv])
        print(f"[mult256] sigma={sig[p]} vel rel err vs oracle {err:.2e}", flush=True)
        assert err <= 1e-8
    B.close()
