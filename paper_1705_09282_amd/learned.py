"""Learned per-level smoothing parameters of the V-cycle.

The smoother's damping eta (equation ASM, eta in (0,1)) and the number of
smoothing steps are predicted per smoothed level by the library's perceptron
(``dfmg_mlp_*``, FP32 HIP kernels).  This module generates the training data
with the method itself and trains the network on the GPU:

* ``step_costs``: a per-cycle time model of the FP32 refinement on a batch
  of four problems of one mesh, t(s) = A + sum_l s_l B_l for s_l smoothing
  steps before and after the coarse correction on level l, from device
  timings of the level kernels and of whole refinement steps.
* ``best_steps``: per training problem, the best uniform count s in 1..6,
  then a coordinate search over s_l (finest first, two passes) minimising
  the modelled time to 1e-8, cycles(s) * t(s), with cycles from the
  contraction of a whole solve.

* ``best_damping``: with those steps, a batch of identical copies solves
  the manufactured load from U = 0 to relative residual 1e-8; every copy
  carries one candidate damping vector, so one batched solve scores all
  candidates.  A coordinate search (finest level first, two
  passes, multiplicative steps around the fixed damping) keeps the per-level
  dampings with the smallest mean contraction per cycle
  rho = (||r_m|| / ||r_0||)^(1/m) over the whole solve.  The target is the
  logit of the best dampings and the best step counts; the fixed damping's
  worst single-cycle ratio (V(2,2)) is kept for the fallback check.
* ``train``: full-batch Adam on the weighted squared error of the outputs
  with the library's forward/backward/Adam kernels.

``python -m paper_1705_09282_amd.learned [out.json]`` runs both on the
default training grid and writes the weights, the training data and the
fallback thresholds (default: ``data/damping_mlp.json`` beside this module).

Chebyshev schedule (``--chebyshev``, default output
``data/chebyshev_mlp.json``): the same network predicts, per smoothed level,
the logit of 1 / alpha (the ratio of the ends of the Chebyshev interval
[b / alpha, b] of the damping schedule) and the smoothing steps.  Targets per
training problem, with the schedule on: ``best_steps`` as above, then a
coordinate search of alpha per level over ``ALPHAS`` (copies of the problem
in one batch, each with its own ratios), scored by the mean contraction per
cycle; the fallback threshold is the fixed damping's, as above.
"""
import json
import math
import os
import sys
import time

import numpy as np

from .dfmg import BatchSolver, Solver, MLP_NPARAM, MLP_NOUT, mlp_adam, mlp_grad, mlp_forward

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "damping_mlp.json")
CHEB_WEIGHTS = os.path.join(HERE, "data", "chebyshev_mlp.json")
ALPHAS = (5.0, 7.0, 10.0, 14.0, 20.0, 30.0)
CHEB_ALPHA0 = 10.0
NOUT = MLP_NOUT   # 5 damping logits, then 5 step counts (finest level first)
NETA = 5
FACTORS = (0.55, 0.7, 0.85, 1.0, 1.15, 1.3, 1.45)
STEPS = (1, 2, 3, 4, 5, 6)
COUNT_WEIGHT = 0.25  # loss weight of a step-count output relative to a logit


def manufactured_speed(d):
    """max |u| of the manufactured velocity (u = curl of the sin^2 potential)
    on the uniform sample grid the library uses (401^2 in 2D, 81^3 in 3D)."""
    m = 400 if d == 2 else 80
    t = np.linspace(0.0, 1.0, m + 1)
    s, ds = np.sin(np.pi * t) ** 2, np.pi * np.sin(2 * np.pi * t)
    if d == 2:
        ux = s[None, :] * ds[:, None]          # [y, x]: s(x) s'(y)
        uy = -ds[None, :] * s[:, None]
        return float(np.sqrt(ux ** 2 + uy ** 2).max())
    X, Y, Z = np.meshgrid(range(m + 1), range(m + 1), range(m + 1), indexing="ij")
    ux = s[X] * ds[Y] * s[Z]
    uy = s[X] * s[Y] * ds[Z] - ds[X] * s[Y] * s[Z]
    return float(np.sqrt(2 * ux ** 2 + uy ** 2).max())


def features(nu, sigma, c, N, k, adv_kind=None, d=2):
    """(log10 nu / 2, log10 sigma / 4, |a| h / nu, k - 1.5) with |a| = max |a|:
    c / sqrt(2) for the rotation, c max|u| for the manufactured velocity."""
    amag = abs(c) * manufactured_speed(d) if adv_kind == 2 else abs(c) / math.sqrt(2.0)
    return np.array([math.log10(nu) / 2.0, math.log10(sigma) / 4.0, amag / (N * nu), k - 1.5], dtype=np.float64)


def logit(p):
    return math.log(p / (1.0 - p))


def contraction(stats):
    """Mean contraction per cycle over the recorded residual history."""
    h = stats["history"]
    if len(h) < 2 or not all(np.isfinite(h)) or h[0] <= 0:
        return float("inf")
    return (h[-1] / h[0]) ** (1.0 / (len(h) - 1))


def worst_cycle(stats):
    """Largest single-cycle ratio ||r_{c}|| / ||r_{c-1}|| for c >= 2, the
    quantity the solver's fallback check compares."""
    h = stats["history"]
    return max(h[c] / h[c - 1] for c in range(2, len(h))) if len(h) > 2 else float("inf")


def score(batch, F, U, etas, tol):
    """Per batch member (each with its own damping vector): the stats of a
    solve from U = 0 to the relative residual tol."""
    batch.set_eta(np.asarray(etas, dtype=np.float64).ravel())
    U.zero_()
    return batch.solve(F, U, tol=tol, raise_on_error=False)


def step_costs(d, N, L, k, device="cuda", reps=20):
    """Per-cycle time model (A, B) of the FP32 refinement for a batch of four
    problems on this mesh: t(s) = A + B . s (B finest level first, ms)."""
    import torch
    m = 12
    S = BatchSolver(d, N, L, k, [1.0] * 4, [1.0] * 4, precision=1, max_cycles=m).bind(device)
    S.autotune(reps=5)
    F = torch.tensor(S.manufactured_rhs(), device=device)
    U = torch.zeros_like(F)
    S.solve(F, U, tol=1e-30, raise_on_error=False)
    Bc = np.array([2.0 * (S.time_kernel(1, lev, reps) + S.time_kernel(3, lev, reps)) for lev in range(L - 1, 0, -1)])
    S.set_smoothing([1] * (L - 1), [1] * (L - 1))
    best = float("inf")
    for _ in range(3):
        U.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.solve(F, U, tol=1e-30, raise_on_error=False)
        torch.cuda.synchronize()
        best = min(best, 1e3 * (time.perf_counter() - t0) / max(1, max(x["cycles"] for x in st)))
    S.close()
    return max(best - Bc.sum(), 0.0), Bc


def best_steps(prob, cost, max_cycles=80, passes=2, tol=1e-8, device="cuda", chebyshev=False):
    """Search of the per-level smoothing steps (pre = post) for one problem
    minimising the modelled solve time cycles(s) * (A + B . s): the best
    uniform count, then coordinate steps; a candidate replaces the current
    steps only if 1% faster.  chebyshev: with the damping schedule at the
    ratio CHEB_ALPHA0.  Returns (steps, modelled ms, contraction)."""
    import torch
    A, Bc = cost
    S = Solver(prob["d"], prob["N"], prob["L"], prob["k"], nu=prob["nu"], sigma=prob["sigma"], c=prob["c"],
               precision=1, max_cycles=max_cycles).bind(device)
    if chebyshev:
        S.set_chebyshev(CHEB_ALPHA0)
    F = torch.tensor(S.manufactured_rhs(), device=device)
    U = torch.zeros_like(F)

    def model(s):
        S.set_smoothing(s, s)
        U.zero_()
        rho = contraction(S.solve(F, U, tol=tol, raise_on_error=False))
        if not rho < 1.0:
            return float("inf"), rho
        return (A + float(Bc @ np.asarray(s))) * math.log(tol) / math.log(max(rho, 1e-12)), rho

    nlev = prob["L"] - 1
    # uniform counts first (a single level's count alone moves little when
    # the others limit the contraction), then per-level refinement
    best, cur, rho = float("inf"), [2] * nlev, float("inf")
    for v in STEPS:
        t, r = model([v] * nlev)
        if t < best:
            best, cur, rho = t, [v] * nlev, r
    for _ in range(passes):
        for lev in range(nlev):
            for v in STEPS:
                if v == cur[lev]:
                    continue
                cand = list(cur)
                cand[lev] = v
                t, r = model(cand)
                if t < 0.99 * best:
                    best, cur, rho = t, cand, r
    S.close()
    return cur, best, rho


def best_damping(prob, steps=None, max_cycles=80, passes=2, tol=1e-8, device="cuda"):
    """Coordinate search of the per-level damping for one problem: every
    candidate is scored by the mean contraction per cycle of a whole solve to
    tol from U = 0 (the quantity that sets the cost of a solve); a candidate
    replaces the current dampings only if it contracts at least 1% faster.
    prob: dict(d, N, k, L, nu, sigma, c); steps: per-level smoothing steps
    (finest first; None: the default V(2,2)).  Returns (eta_best, rho_best,
    rho_plain, worst single-cycle ratio of the fixed damping with V(2,2))."""
    import torch
    C = len(FACTORS)
    B = BatchSolver(prob["d"], prob["N"], prob["L"], prob["k"], [prob["nu"]] * C, [prob["sigma"]] * C,
                    [prob["c"]] * C, precision=1, max_cycles=max_cycles).bind(device)
    F = torch.tensor(B.manufactured_rhs(), device=device)
    U = torch.zeros_like(F)
    eta0 = B.get_eta()[0].copy()
    nlev = eta0.size
    cur = eta0.copy()
    st = score(B, F, U, [eta0] * C, tol)[0]
    rho_plain, worst_plain = contraction(st), worst_cycle(st)
    if steps is not None:
        B.set_smoothing(steps, steps)
        st = score(B, F, U, [eta0] * C, tol)[0]
    best = contraction(st)
    for _ in range(passes):
        for lev in range(nlev):
            cand = []
            for f in FACTORS:
                e = cur.copy()
                e[lev] = min(0.95, cur[lev] * f)
                cand.append(e)
            rho = np.array([contraction(x) for x in score(B, F, U, cand, tol)])
            i = int(np.argmin(rho))
            if rho[i] < 0.99 * best:
                best, cur = rho[i], cand[i]
    B.close()
    return cur, best, rho_plain, worst_plain


def best_alpha(prob, steps, max_cycles=80, passes=1, tol=1e-8, device="cuda"):
    """Coordinate search of the schedule's ratio alpha per level for one
    problem with the given steps: copies of the problem in one batch, copy j
    with ALPHAS[j] on the level searched; the candidate with the smallest
    mean contraction per cycle replaces the current ratios if 1% better.
    Returns (alphas, rho_best, rho_plain, worst single-cycle ratio of the
    fixed damping with V(2,2))."""
    import torch
    C = len(ALPHAS)
    B = BatchSolver(prob["d"], prob["N"], prob["L"], prob["k"], [prob["nu"]] * C, [prob["sigma"]] * C,
                    [prob["c"]] * C, precision=1, max_cycles=max_cycles).bind(device)
    F = torch.tensor(B.manufactured_rhs(), device=device)
    U = torch.zeros_like(F)
    U.zero_()
    st = B.solve(F, U, tol=tol, raise_on_error=False)[0]
    rho_plain, worst_plain = contraction(st), worst_cycle(st)
    B.set_smoothing(steps, steps)
    B.set_chebyshev(CHEB_ALPHA0)
    nlev = prob["L"] - 1
    cur = np.full(nlev, CHEB_ALPHA0)

    def scores(cands):
        B.set_chebyshev_alpha(np.array(cands))
        U.zero_()
        return np.array([contraction(x) for x in B.solve(F, U, tol=tol, raise_on_error=False)])

    best = scores([cur] * C)[0]
    for _ in range(passes):
        for lev in range(nlev):
            cand = []
            for a in ALPHAS:
                e = cur.copy()
                e[lev] = a
                cand.append(e)
            rho = scores(cand)
            i = int(np.argmin(rho))
            if rho[i] < 0.99 * best:
                best, cur = rho[i], cand[i]
    B.close()
    return cur, best, rho_plain, worst_plain


def training_problems():
    """Default training grid: 2D, both degrees, 128^2 with 6 grids over
    nu x sigma x |a|h/nu, plus the Stokes problems of both degrees on 256^2."""
    out = []
    for k in (1, 2):
        for nu in (1.0, 0.1, 0.01):
            for sigma in (1e-2, 1.0, 1e2, 1e4):
                for peh in (0.0, 0.25, 0.5, 0.75, 1.0):
                    c = math.sqrt(2.0) * nu * 128 * peh
                    out.append(dict(d=2, N=128, k=k, L=6, nu=nu, sigma=sigma, c=c))
                out.append(dict(d=2, N=256, k=k, L=6, nu=nu, sigma=sigma, c=0.0))
    return out


def sweep(problems, log=None, chebyshev=False):
    """Training data: X (n x 4), Y (n x 10) targets (damping logits, step
    counts; chebyshev: logits of 1 / alpha, step counts), M (n x 10)
    weights, rho_plain, rho_best, worst_plain, steps, and the time model of
    every mesh."""
    X, Y, Mk, rp, rb, wp, ss = [], [], [], [], [], [], []
    costs = {}
    for i, p in enumerate(problems):
        t0 = time.time()
        key = (p["d"], p["N"], p["L"], p["k"])
        if key not in costs:
            costs[key] = step_costs(*key)
            if log:
                log(f"[sweep] time model {key}: A {costs[key][0]:.4f} ms, B {np.round(costs[key][1], 4).tolist()}")
        steps, ms, rho_s = best_steps(p, costs[key], passes=1 if chebyshev else 2, chebyshev=chebyshev)
        if chebyshev:
            alpha, rho, rho_plain, worst = best_alpha(p, steps)
            eta = 1.0 / alpha   # the network's first outputs: logit of a / b
        else:
            eta, rho, rho_plain, worst = best_damping(p, steps)
        y = np.zeros(NOUT)
        mk = np.zeros(NOUT)
        for j in range(min(NETA, eta.size)):
            y[j] = logit(eta[j])
            mk[j] = 1.0
            y[NETA + j] = steps[j]
            mk[NETA + j] = COUNT_WEIGHT
        X.append(features(p["nu"], p["sigma"], p["c"], p["N"], p["k"]))
        Y.append(y)
        Mk.append(mk)
        rp.append(rho_plain)
        rb.append(rho)
        wp.append(worst)
        ss.append(steps[:NETA])
        if log:
            what = f"alpha {np.round(1.0 / eta, 1).tolist()}" if chebyshev else f"eta {np.round(eta, 3).tolist()}"
            log(f"[sweep {i + 1}/{len(problems)}] {p} steps {steps} (model {ms:.2f} ms) rho plain {rho_plain:.3f} "
                f"-> {rho:.3f} {what} ({time.time() - t0:.1f} s)")
    return dict(X=np.array(X), Y=np.array(Y), M=np.array(Mk), rho_plain=np.array(rp), rho_best=np.array(rb),
                worst_plain=np.array(wp), steps=np.array(ss),
                time_model=np.array([[*k, c[0], *c[1]] for k, c in costs.items()]))


def glorot_init(seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    shapes = [(32, 4), (32,), (32, 32), (32,), (NOUT, 32), (NOUT,)]
    parts = []
    for shp in shapes:
        if len(shp) == 2:
            lim = math.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts).astype(np.float32)


def train(X, Y, M, epochs=3000, lr=3e-3, seed=0, device="cuda", log=None):
    """Full-batch Adam with the library's kernels; returns (W, loss history)."""
    import torch
    n = X.shape[0]
    W = torch.tensor(glorot_init(seed), device=device)
    # start the output bias at the mean target of each output
    ymean = (Y * M).sum(axis=0) / np.maximum(M.sum(axis=0), 1)
    W[MLP_NPARAM - NOUT:] = torch.tensor(ymean, dtype=torch.float32, device=device)
    Xd = torch.tensor(X, dtype=torch.float32, device=device).contiguous()
    Yd = torch.tensor(Y, dtype=torch.float32, device=device).contiguous()
    Md = torch.tensor(M, dtype=torch.float32, device=device).contiguous()
    m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=device)
    v = torch.zeros_like(m)
    G = torch.zeros_like(m)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    work = torch.zeros(n * (MLP_NPARAM + 1), dtype=torch.float32, device=device)
    scale = 1.0 / float(M.sum())
    hist = []
    for t in range(1, epochs + 1):
        mlp_grad(W, Xd, Yd, Md, scale, work, G, loss)
        mlp_adam(W, m, v, G, t, lr)
        if t % 100 == 0 or t == 1:
            hist.append((t, float(loss.item())))
            if log and t % 500 == 0:
                log(f"[train] epoch {t} loss {hist[-1][1]:.5f}")
    mlp_grad(W, Xd, Yd, Md, scale, work, G, loss)
    hist.append((epochs + 1, float(loss.item())))
    return W.cpu().numpy(), hist


def predict(W, X, device="cuda"):
    import torch
    Wd = torch.tensor(np.asarray(W, dtype=np.float32), device=device)
    Xd = torch.tensor(np.asarray(X, dtype=np.float32), device=device).contiguous()
    Z = torch.zeros(X.shape[0] * NOUT, dtype=torch.float32, device=device)
    mlp_forward(Wd, Xd, Z)
    return Z.cpu().numpy().reshape(-1, NOUT)


def save(path, W, data, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    out = {"W": [float(x) for x in W], "meta": meta,
           "train": {k: np.asarray(v).tolist() for k, v in data.items()}}
    with open(path, "w") as f:
        json.dump(out, f)


def load(path=WEIGHTS):
    d = json.load(open(path))
    d["W"] = np.array(d["W"], dtype=np.float32)
    for k, v in d["train"].items():
        d["train"][k] = np.array(v)
    return d


def rho_plain_for(model, feats, neighbours=8):
    """Fallback threshold: the largest worst single-cycle ratio of the fixed
    damping over the nearest training points (feature space).  Taking the
    largest keeps the check from firing on problems that merely lie between
    training points; weights that stall or diverge still exceed it."""
    X = model["train"]["X"]
    rp = model["train"]["worst_plain"]
    out = []
    for f in np.atleast_2d(feats):
        near = np.argsort(((X - f) ** 2).sum(axis=1))[:neighbours]
        out.append(float(rp[near].max()))
    return np.array(out)


def problem_features(solver):
    """Network inputs of every problem of a Solver, BatchSolver or
    MultiSolver (whose problems have their own grids and degrees)."""
    kind = getattr(solver, "adv_kind", None)
    if hasattr(solver, "meshes"):
        return np.array([features(nu, sg, c, m[1], m[3], kind, m[0])
                         for nu, sg, c, m in zip(solver.nus, solver.sigmas, solver.cs, solver.meshes)])
    return np.array([features(nu, sg, c, solver.n_elem, solver.k, kind, solver.dim)
                     for nu, sg, c in zip(solver.nus, solver.sigmas, solver.cs)])


def measured_worst_plain(solver, tol=1e-8, seed=0):
    """Fallback thresholds measured on the problems themselves: the worst
    single-cycle residual ratio (cycles 2 on) of a solve with the fixed
    damping from U = 0 to tol, with a seeded random velocity load (pressure
    rows zero), in the solver's own precision -- the quantity the training
    sweep records per training problem.  Leaves the solver on the fixed
    damping."""
    import torch
    solver.set_learned(None)
    solver.set_learned_chebyshev(None)
    n, P = solver.n, solver.nprob
    nv = solver.sizes()["n_vel"]
    F = np.random.default_rng(seed).uniform(-1.0, 1.0, (P, n))
    F[:, nv:] = 0.0
    F = torch.tensor(F.ravel(), device=solver._ws.device)
    U = torch.zeros_like(F)
    st = solver._solve(F, U, tol, False)
    return np.array([worst_cycle(x) for x in st])


def fallback_thresholds(model, solver):
    """Per problem: the threshold of the nearest training points (2D, unit
    square), or the measured one where the features do not describe the
    problem and its plain rate differs: a mapped domain, or a 3D problem of a
    Solver or BatchSolver."""
    if getattr(solver, "geometry", 0) or (not hasattr(solver, "meshes") and getattr(solver, "dim", 2) == 3):
        return measured_worst_plain(solver)
    return rho_plain_for(model, problem_features(solver))


def apply(solver, model=None, fallback=True):
    """Switch a bound Solver/BatchSolver/MultiSolver to the learned dampings of `model`
    (default: the shipped weights), with the fallback thresholds of
    fallback_thresholds().  A model trained with --chebyshev sets the
    learned Chebyshev schedule instead."""
    model = load() if model is None else model
    rho = fallback_thresholds(model, solver) if fallback else None
    if model["meta"].get("mode") == "chebyshev":
        solver.set_learned_chebyshev(model["W"], rho)
    else:
        solver.set_learned(model["W"], rho)


def apply_chebyshev(solver, model=None, fallback=True):
    """apply() with the shipped Chebyshev-schedule network by default."""
    apply(solver, load(CHEB_WEIGHTS) if model is None else model, fallback)


def main():
    log = lambda s: print(s, flush=True)
    args = [a for a in sys.argv[1:] if a != "--chebyshev"]
    cheb = "--chebyshev" in sys.argv[1:]
    t0 = time.time()
    probs = training_problems()
    data = sweep(probs, log=log, chebyshev=cheb)
    log(f"[sweep] {len(probs)} problems in {time.time() - t0:.0f} s; mean rho plain "
        f"{data['rho_plain'].mean():.3f} best {data['rho_best'].mean():.3f}")
    W, hist = train(data["X"], data["Y"], data["M"], log=log)
    meta = {"epochs": hist[-1][0] - 1, "final_loss": hist[-1][1], "factors": FACTORS,
            "objective": "steps: modelled time to 1e-8 of the FP32 refinement (4-problem batch); dampings: "
                         "mean contraction per cycle of a solve to 1e-8 from U=0 with those steps",
            "problems": len(probs), "features": "log10(nu)/2, log10(sigma)/4, |a|h/nu, k-1.5"}
    if cheb:
        meta.update(mode="chebyshev", alphas=ALPHAS,
                    objective="steps: modelled time to 1e-8 of the FP32 refinement with the Chebyshev schedule "
                              f"(alpha {CHEB_ALPHA0}); alpha per level: mean contraction per cycle of a solve to "
                              "1e-8 from U=0 with those steps; outputs 0..4 are logit(1/alpha)")
    out = args[0] if args else (CHEB_WEIGHTS if cheb else WEIGHTS)
    save(out, W, data, meta)
    log(f"[train] final loss {hist[-1][1]:.5f}; wrote {out}")


if __name__ == "__main__":
    sys.exit(main())
