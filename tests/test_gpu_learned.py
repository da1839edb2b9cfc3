"""Learned per-level damping on the GPU: the network kernels against the FP64
oracle, the dampings a solver derives from a network, V-cycles with those
dampings against the oracle, training, the shipped model on held-out
problems and the fallback to the fixed damping.

Tolerances: the network runs in FP32; logits of O(1) agree with the FP64
oracle (evaluated on the same FP32-rounded weights and inputs) to ~1e-6, so
1e-5 absolute is used; gradients (sums over samples in FP32) to 1e-4 of their
largest entry."""
import math
import os

import numpy as np
import pytest

from oracle import mlp as om
from oracle.multigrid import Hierarchy, vcycles
from oracle.assemble import load_vector, rotation_field
from oracle.manufactured import forcing

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def tdev(x):
    return torch.tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


def sample_data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, (n, om.NIN))
    Y = rng.normal(0.0, 1.0, (n, om.NOUT))
    M = (rng.uniform(size=(n, om.NOUT)) < 0.8).astype(np.float64)
    M[0] = 1.0
    return X, Y, M


def weights(seed):
    rng = np.random.default_rng(seed + 100)
    return f32(om.init(seed) + rng.normal(0.0, 0.1, om.NPARAM))


def test_forward_matches_oracle():
    from paper_1705_09282_amd.dfmg import mlp_forward
    for n in (1, 63, 64, 200):
        W = weights(n)
        X, _, _ = sample_data(n, n)
        X = f32(X)
        Z = torch.zeros(n * om.NOUT, dtype=torch.float32, device="cuda")
        mlp_forward(tdev(W), tdev(X), Z)
        ref = om.forward(W, X)
        err = np.max(np.abs(Z.cpu().numpy().reshape(n, om.NOUT) - ref))
        print(f"[forward] n={n} max err {err:.2e}", flush=True)
        assert err < 1e-5


def test_grad_and_loss_match_oracle():
    from paper_1705_09282_amd.dfmg import mlp_grad, MLP_NPARAM
    for n in (1, 50, 130):
        W = weights(n + 1)
        X, Y, M = sample_data(n, n + 7)
        X, Y = f32(X), f32(Y)
        G = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        work = torch.zeros(n * (MLP_NPARAM + 1), dtype=torch.float32, device="cuda")
        scale = float(np.float32(1.0 / M.sum()))
        mlp_grad(tdev(W), tdev(X), tdev(Y), tdev(M), scale, work, G, loss)
        g_ref = om.grad(W, X, Y, M) * (scale * M.sum())
        l_ref = om.loss(W, X, Y, M) * (scale * M.sum())
        g = G.cpu().numpy().astype(np.float64)
        gerr = np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))
        lerr = abs(float(loss.item()) - l_ref) / l_ref
        print(f"[grad] n={n} grad rel err {gerr:.2e} loss rel err {lerr:.2e}", flush=True)
        assert gerr < 1e-4 and lerr < 1e-5


def test_grad_is_deterministic():
    from paper_1705_09282_amd.dfmg import mlp_grad, MLP_NPARAM
    n = 300
    W = weights(5)
    X, Y, M = sample_data(n, 9)
    out = []
    for _ in range(2):
        G = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        work = torch.zeros(n * (MLP_NPARAM + 1), dtype=torch.float32, device="cuda")
        mlp_grad(tdev(W), tdev(X), tdev(Y), tdev(M), 0.01, work, G, loss)
        out.append(np.concatenate([G.cpu().numpy(), loss.cpu().numpy()]))
    assert np.array_equal(out[0], out[1])


def test_adam_matches_oracle():
    from paper_1705_09282_amd.dfmg import mlp_adam, MLP_NPARAM
    rng = np.random.default_rng(11)
    W = f32(rng.normal(size=MLP_NPARAM))
    m = f32(rng.normal(scale=0.1, size=MLP_NPARAM))
    v = f32(rng.uniform(0.0, 0.1, size=MLP_NPARAM))
    G = f32(rng.normal(size=MLP_NPARAM))
    for t in (1, 7):
        Wd, md, vd = tdev(W), tdev(m), tdev(v)
        mlp_adam(Wd, md, vd, tdev(G), t, 3e-3)
        Wr, mr, vr = om.adam_step(W, G, m, v, t, lr=3e-3)
        for a, b, name in ((Wd, Wr, "W"), (md, mr, "m"), (vd, vr, "v")):
            err = np.max(np.abs(a.cpu().numpy() - b) / (1.0 + np.abs(b)))
            assert err < 2e-6, (t, name, err)


def test_training_follows_oracle_and_reduces_loss():
    """Full-batch Adam on a smooth target: the first steps track the FP64
    oracle's trajectory; after 600 steps the loss has dropped tenfold."""
    from paper_1705_09282_amd import learned
    from paper_1705_09282_amd.dfmg import mlp_grad, mlp_adam, MLP_NPARAM
    rng = np.random.default_rng(21)
    n = 80
    X = f32(rng.uniform(-1, 1, (n, om.NIN)))
    Y = f32(np.stack([np.sin(X[:, 0] + o * 0.3) + 0.5 * X[:, 1] * X[:, 2] - 0.2 * o for o in range(om.NOUT)], 1))
    M = np.ones((n, om.NOUT))
    W0 = f32(learned.glorot_init(4))
    Wd = tdev(W0)
    md = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
    vd = torch.zeros_like(md)
    G = torch.zeros_like(md)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = torch.zeros(n * (MLP_NPARAM + 1), dtype=torch.float32, device="cuda")
    Xd, Yd, Md = tdev(X), tdev(Y), tdev(M)
    scale = 1.0 / M.sum()
    Wr, mr, vr = W0.copy(), np.zeros(MLP_NPARAM), np.zeros(MLP_NPARAM)
    l0 = om.loss(W0, X, Y, M)
    for t in range(1, 601):
        mlp_grad(Wd, Xd, Yd, Md, scale, work, G, loss)
        mlp_adam(Wd, md, vd, G, t, 1e-2)
        if t <= 5:
            Wr, mr, vr = om.adam_step(Wr, om.grad(Wr, X, Y, M), mr, vr, t, lr=1e-2)
            err = np.max(np.abs(Wd.cpu().numpy() - Wr))
            assert err < 1e-4, (t, err)
    l_end = om.loss(Wd.cpu().numpy().astype(np.float64), X, Y, M)
    print(f"[train] loss {l0:.4f} -> {l_end:.5f}", flush=True)
    assert l_end < 0.1 * l0


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


@pytest.mark.parametrize("N,L,k", [(16, 3, 1), (64, 6, 2), (128, 7, 1)])
def test_solver_dampings_are_the_network_output(N, L, k):
    """Per problem of a batch, eta of the finest smoothed level first equals
    sigmoid of the oracle network's damping outputs on the problem's
    features, and the batch's smoothing steps are the largest rounded count
    output over its problems; levels beyond the five outputs reuse the last
    one.  Without a network the fixed damping and V(2,2) come back."""
    from paper_1705_09282_amd.dfmg import BatchSolver
    nus, sigmas, cs = [1.0, 0.1, 0.02], [1e-2, 30.0, 1e4], [0.0, 3.0, 1.5]
    print(f"\n[case] N={N} L={L} k={k}", flush=True)
    B = BatchSolver(2, N, L, k, nus, sigmas, cs).bind()
    W = weights(2)
    fixed = B.get_eta()
    B.set_learned(W)
    eta = B.get_eta()
    X = np.array([om.features(nu, sg, abs(c) / math.sqrt(2.0), N, k) for nu, sg, c in zip(nus, sigmas, cs)])
    Z = om.forward(W, f32(X))
    for p in range(3):
        ref = [sigmoid(Z[p, min(i, om.NETA - 1)]) for i in range(L - 1)]
        assert np.max(np.abs(eta[p] - ref)) < 1e-5
    steps = om.steps(Z[:, om.NETA:]).max(axis=0)
    ref = [int(steps[min(i, om.NETA - 1)]) for i in range(L - 1)]
    assert B.get_smoothing() == (ref, ref)
    B.set_learned(None)
    assert np.array_equal(B.get_eta(), fixed)
    assert B.get_smoothing() == ([2] * (L - 1), [2] * (L - 1))
    B.close()


def test_vcycles_with_learned_dampings_match_oracle():
    from paper_1705_09282_amd.dfmg import Solver
    d, N, k, L, nu, sigma, c = 2, 16, 2, 3, 0.1, 10.0, 2.0
    print(f"\n[case] N={N} L={L} k={k} nu={nu} sigma={sigma} c={c}", flush=True)
    s = Solver(d, N, L, k, nu=nu, sigma=sigma, c=c).bind()
    W = weights(6)
    s.set_learned(W)
    eta = s.get_eta()[0]
    adv = rotation_field(c)
    h = Hierarchy(d, N, k, L, nu, sigma, adv)
    F = load_vector(h.finest.disc, forcing(d, nu, sigma, adv))
    Fd = torch.tensor(F, device="cuda")
    U = torch.zeros_like(Fd)
    s.vcycle(Fd, U, 3)
    n1, n2 = s.get_smoothing()
    ref = vcycles(h, np.zeros_like(F), F, 3, nu1=n1, nu2=n2, eta=list(eta))
    got = U.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"[vcycles] eta {np.round(eta, 4).tolist()} rel err {err:.2e}", flush=True)
    assert err < 1e-10
    s.close()


HELD_OUT = [(2, 128, 6, 2, 0.3, 10.0, 0.25), (2, 128, 6, 1, 0.03, 1e3, 0.0), (2, 128, 6, 2, 1.0, 0.1, 0.75),
            (2, 256, 6, 1, 0.3, 3e2, 0.5), (2, 256, 6, 2, 0.03, 3.0, 0.25)]


def test_learned_beats_fixed_on_held_out_problems():
    """The shipped model against the fixed damping, to relative residual
    1e-8, on parameters outside the training grid: no problem needs more than
    one extra cycle and the total drops; both solutions stay
    divergence-free."""
    from paper_1705_09282_amd import learned
    from paper_1705_09282_amd.dfmg import BatchSolver
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("no trained damping model")
    model = learned.load()
    tot = {"fixed": 0, "learned": 0}
    for (d, N, L, k, nu, sigma, peh) in HELD_OUT:
        c = math.sqrt(2.0) * nu * N * peh
        print(f"\n[case] N={N} L={L} k={k} nu={nu} sigma={sigma} Pe_h={peh}", flush=True)
        B = BatchSolver(d, N, L, k, [nu], [sigma], [c], max_cycles=100).bind()
        F = torch.tensor(B.manufactured_rhs(), device="cuda")
        cyc = {}
        for mode in ("fixed", "learned"):
            if mode == "learned":
                learned.apply(B, model)
                print(f"[learned] predicted eta {np.round(B.get_eta()[0], 3).tolist()}", flush=True)
            U = torch.zeros_like(F)
            st = B.solve(F, U, tol=1e-8)[0]
            div = B.div_norm(U)[0]
            cyc[mode] = st["cycles"]
            tot[mode] += st["cycles"]
            print(f"[{mode}] eta {np.round(B.get_eta()[0], 3).tolist()} cycles {st['cycles']} "
                  f"fallback {st['fallback']} div {div:.1e}", flush=True)
            assert st["converged"] and div < 1e-10
        assert cyc["learned"] <= cyc["fixed"] + 1
        B.close()
    assert tot["learned"] < tot["fixed"]


@pytest.mark.parametrize("bias", [-12.0, 8.0])
def test_fallback_under_extreme_weights(bias):
    """Weights that drive every damping to ~0 (no smoothing) or ~1 (an
    unstable smoother): the check switches to the fixed damping, the solve
    converges, and the next solve starts from the learned dampings again."""
    from paper_1705_09282_amd.dfmg import Solver
    from paper_1705_09282_amd import learned
    N, L, k = 64, 5, 1
    s = Solver(2, N, L, k, nu=1.0, sigma=1.0, max_cycles=200).bind()
    F = torch.tensor(s.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    fixed = s.get_eta()
    st0 = s.solve(F, U, tol=1e-8)
    rho = learned.worst_cycle(st0)
    W = np.zeros(om.NPARAM, dtype=np.float32)
    W[om.NPARAM - om.NOUT:om.NPARAM - om.NOUT + om.NETA] = bias
    W[om.NPARAM - om.NOUT + om.NETA:] = 2.0  # V(2,2)
    s.set_learned(W, [rho])
    assert np.allclose(s.get_eta(), sigmoid(bias), atol=1e-6)
    for rep in range(2):
        U.zero_()
        st = s.solve(F, U, tol=1e-8)
        print(f"[fallback] bias {bias} rep {rep} cycles {st['cycles']} (fixed {st0['cycles']}) "
              f"fallback {st['fallback']}", flush=True)
        assert st["converged"] and st["fallback"]
        assert np.array_equal(s.get_eta(), fixed)
        assert s.div_norm(U) < 1e-10
        assert s.residual_norm(F, U) <= 1e-8 * st["fnorm"] * 1.0001
    s.close()


def test_no_fallback_without_threshold():
    """Without a plain rate the learned dampings are kept for the whole solve,
    also after a solve that did fall back (the thresholds live on the device,
    so the captured cycle graph follows them)."""
    from paper_1705_09282_amd.dfmg import Solver
    s = Solver(2, 32, 4, 1, nu=1.0, sigma=1.0, max_cycles=60).bind()
    F = torch.tensor(s.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    W = np.zeros(om.NPARAM, dtype=np.float32)
    W[om.NPARAM - om.NOUT:om.NPARAM - om.NOUT + om.NETA] = math.log(0.3 / 0.7)
    W[om.NPARAM - om.NOUT + om.NETA:] = 2.0
    s.set_learned(W, [1e-6])  # any cycle contracts worse than this
    st = s.solve(F, U, tol=1e-8)
    assert st["converged"] and st["fallback"]
    s.set_learned(W)
    U.zero_()
    st = s.solve(F, U, tol=1e-8)
    assert st["converged"] and not st["fallback"]
    assert np.allclose(s.get_eta(), 0.3, atol=1e-6)
    s.set_learned(None)
    U.zero_()
    st = s.solve(F, U, tol=1e-8)
    assert st["converged"] and not st["fallback"]
    s.close()
