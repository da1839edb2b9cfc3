#!/usr/bin/env python3
"""Throughput of the divergence-conforming multigrid solver on one MI355X.

Workload (synthetic, seeded): 2D generalized Stokes on the unit square,
pressure degree k=2 (velocity S^{3,2} x S^{2,3}), 256x256 elements, 6 grids
(256 .. 8), nu = 1, sigma in {1e-2, 1, 1e2, 1e4}, load vector of the
manufactured solution u = curl(sin^2(pi x) sin^2(pi y)), p = sin(2 pi x)
sin(2 pi y).  One step solves all four problems from U = 0 to relative
residual 1e-8; inputs are resident in HBM before timing.  The timed path is
the learned Chebyshev damping schedule (the network predicts per level the
schedule's interval ratio and the smoothing steps) with FP32 V-cycles inside
FP64 iterative refinement.  Timed beside it on the same problems: the plain
FP64 solver (fixed damping, V(2,2)), FP32 refinement with the fixed damping
and V(2,2), FP32 refinement with the learned constant per-level damping and
steps, the learned schedule in plain FP64 cycles, and the paper's
multiplicative Schwarz smoother with V(1,2) in FP64 cycles.

Prints one JSON line: metric, value (DOF/s over the whole step, DOFs =
dim V_h + dim Q_h), roofline of the dominant kernel (finest-grid residual
SpMV), and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF/s solved to 1e-8 rel. residual; learned+FP32-refined vs plain FP64 GPU"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmv_stokes2d_traffic.json")
TRAFFIC_FILE_HBM = os.path.join(ROOT, "profiles", "spmv_stokes2d_1024_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1705_09282_amd", "csrc", f)
               for f in ("spmv.hip", "spmv_dev.hpp", "layout.hpp", "device_util.hpp")]


def kernel_hash():
    """Hash of the residual kernel's sources (the counters stay valid only
    while these are unchanged)."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, path=TRAFFIC_FILE):
    """HBM bytes per launch of a residual kernel from the committed rocprofv3
    counter runs, or None if missing, taken on other kernel code or on
    another workload."""
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    if t.get("workload") != workload:
        return None
    return t.get("bytes_per_launch")


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count()
    return model, ncores


def cpu_baseline(tol, U_gpu, runs=5, warmup=1):
    """The oracle as it stands on one of the four problems (sigma = 1): full
    solves to tol from U = 0, setup excluded as for the GPU; `warmup` untimed
    solves, then the median of `runs`, once with the BLAS/OpenMP pools at one
    thread and once at every core this process may use.  Afterwards the
    oracle continues its solve to 1e-12, and the GPU's sigma = 1 velocity is
    compared with it."""
    import statistics
    from threadpoolctl import threadpool_limits, threadpool_info
    import numpy as np
    import workloads
    from oracle.multigrid import Hierarchy, solve
    from oracle.assemble import load_vector
    from oracle.manufactured import forcing
    model, ncores = host_cpu()
    cfg = workloads.stokes2d(1.0)
    h = Hierarchy(cfg["d"], cfg["N"], cfg["k"], cfg["L"], cfg["nu"], cfg["sigma"])
    F = load_vector(h.finest.disc, forcing(cfg["d"], cfg["nu"], cfg["sigma"]))
    dofs = h.finest.disc.dofs()
    legs = {}
    for name, limit in (("one_core", 1), ("all_cores", ncores)):
        with threadpool_limits(limit):
            threads = max([1] + [p.get("num_threads", 1) for p in threadpool_info()])
            times = []
            for i in range(warmup + runs):
                t0 = time.perf_counter()
                U, hist = solve(h, F, tol=tol)
                if i >= warmup:
                    times.append(time.perf_counter() - t0)
        med = statistics.median(times)
        legs[name] = {"value": dofs / med, "seconds_median": med, "seconds": times, "threads": threads,
                      "cycles": len(hist) - 1}
    Uo, _ = solve(h, F, tol=1e-12, U0=U, max_cycles=400)
    nv = h.finest.disc.n_v
    err = float(np.linalg.norm(U_gpu[:nv] - Uo[:nv]) / np.linalg.norm(Uo[:nv]))
    best = legs["all_cores"]
    return {"value": best["value"], "unit": "DOF/s", "cores": best["threads"], "kind": "oracle",
            "sample": f"sigma=1 problem only (1 of 4): FP64 oracle solves to {tol:g} from U=0, 256x256, k=2, "
                      f"6 grids, V(2,2), setup excluded; median of {runs} after {warmup} warm-up, BLAS/OpenMP "
                      f"pools at every core ({ncores}) and at one",
            "one_core": legs["one_core"], "all_cores": legs["all_cores"],
            "cpu_model": model, "nproc": ncores}, err


def paper_oseen_legs(dev, steps=3, warmup=1):
    """The paper's generalized Oseen problems on the GPU (context, not the
    metric): 2D k=1 (the paper's p = 2), 256^2 elements refined from a
    single coarsest element (9 grids), nu = 1, sigma = Da = 1000, advection
    = the manufactured velocity scaled to max|a| / nu = Re in {1, 100}; the
    two problems as one batch solved from U = 0 to 1e-8, with the
    multiplicative smoother V(1,2) (the paper's) and the additive one V(2,2)
    (fixed damping), FP64."""
    import math
    import torch
    from paper_1705_09282_amd.dfmg import BatchSolver
    from paper_1705_09282_amd.learned import manufactured_speed
    res = [1.0, 100.0]
    cs = [r / manufactured_speed(2) for r in res]
    out = {"workload": "2D generalized Oseen, k=1, 256x256, 9 grids, nu=1, Da=1000, a = manufactured velocity, "
                       "Re in {1, 100}, tol 1e-8, U0=0"}
    for name, opts in (("multiplicative_v12", dict(multiplicative=1, nu1=1, nu2=2)), ("additive_v22", {})):
        b = BatchSolver(2, 256, 9, 1, [1.0, 1.0], [1000.0, 1000.0], cs, adv_kind=2, max_cycles=300, **opts).bind(dev)
        F = torch.tensor(b.manufactured_rhs(), device=dev)
        U = torch.zeros_like(F)
        for _ in range(warmup):
            U.zero_()
            b.solve(F, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            U.zero_()
            st = b.solve(F, U)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        dofs = 2 * (b.n - 1)
        out[name] = {"ms_per_solve": 1e3 * dt, "dofs_per_s": dofs / dt, "cycles_per_re": [x["cycles"] for x in st],
                     "div_norm_per_re": [float(x) for x in b.div_norm(U)]}
        b.close()
    return out


def stokes3d_legs(dev, steps=3, warmup=1):
    """The 3D workload (context, not the metric): 3D generalized Stokes,
    k=1, 32^3 elements, 4 grids, nu = 1, the eight seeded log-uniform sigma
    as one batch, solved from U = 0 to 1e-8: plain FP64 with the fixed
    damping V(2,2), and FP32 V-cycles in FP64 refinement with the Chebyshev
    schedule (3D default ratio, V(6,6)) and autotuned kernels and tiles."""
    import torch
    import workloads
    from paper_1705_09282_amd.dfmg import BatchSolver
    sig = workloads.stokes3d_sigmas()
    out = {"workload": "stokes3d: 3D generalized Stokes, k=1, 32^3, 4 grids, nu=1, 8 seeded sigma in "
                       "[1e-2, 1e4], tol 1e-8, U0=0"}
    for name, prec, sched in (("fp64_fixed_damping", 0, False), ("fp32_refined_chebyshev_v66", 1, True)):
        b = BatchSolver(3, 32, 4, 1, [1.0] * len(sig), list(sig), precision=prec, max_cycles=400).bind(dev)
        b.autotune(reps=10)
        if sched:
            b.set_smoothing([6, 6, 6], [6, 6, 6])
            b.set_chebyshev()
        F = torch.tensor(b.manufactured_rhs(), device=dev)
        U = torch.zeros_like(F)
        for _ in range(warmup):
            U.zero_()
            b.solve(F, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            U.zero_()
            st = b.solve(F, U)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        dofs = len(sig) * (b.n - 1)
        out[name] = {"ms_per_solve": 1e3 * dt, "dofs_per_s": dofs / dt, "cycles_per_sigma": [x["cycles"] for x in st],
                     "max_div_norm": float(b.div_norm(U).max())}
        b.close()
    out["speedup"] = out["fp64_fixed_damping"]["ms_per_solve"] / out["fp32_refined_chebyshev_v66"]["ms_per_solve"]
    return out


def annulus_legs(dev, steps=3, warmup=1):
    """The benchmark's discretization on the paper's quarter annulus
    (context): 2D generalized Stokes, k=2, 256^2 elements, 6 grids, nu = 1,
    the four sigma as one batch, a seeded random velocity load (the paper's
    manufactured solution is defined on the unit square), solved from U = 0
    to 1e-8: FP64 additive with the fixed damping V(2,2), FP64
    multiplicative V(1,2), and FP32 refinement with the learned Chebyshev
    schedule (its fallback thresholds measured by one fixed-damping solve of
    the batch, reported apart); the host setup (quadrature assembly through the Piola maps,
    Galerkin products, per-subdomain inverses) reported apart; the FP32
    residual, whose velocity rows couple both components, timed alone."""
    import torch
    import workloads
    from paper_1705_09282_amd.dfmg import BatchSolver
    from paper_1705_09282_amd import learned
    sig = [1e-2, 1.0, 1e2, 1e4]
    out = {"workload": "quarter annulus r_i=0.075 r_o=0.225, 2D generalized Stokes, k=2, 256^2, 6 grids, nu=1, "
                       "sigma in {1e-2, 1, 1e2, 1e4}, seeded random velocity load, tol 1e-8, U0=0"}
    for name, opt, sched in (("fp64_additive_fixed_damping", {}, False),
                             ("fp64_multiplicative_v12", {"multiplicative": 1, "nu1": 1, "nu2": 2}, False),
                             ("fp32_refined_learned_chebyshev", {"precision": 1}, True)):
        t0 = time.perf_counter()
        b = BatchSolver(2, 256, 6, 2, [1.0] * len(sig), sig, geometry=1, max_cycles=400, **opt).bind(dev)
        setup = time.perf_counter() - t0
        b.autotune(reps=10)
        learned_s = None
        if sched:
            t1 = time.perf_counter()
            learned.apply_chebyshev(b)
            learned_s = time.perf_counter() - t1
        n = b.n
        F = workloads.random_coefficients(len(sig) * n, 91)
        nv = 2 * (256 + 1) * (256 + 2)
        for p in range(len(sig)):
            F[p * n + nv:(p + 1) * n] = 0.0
        F = torch.tensor(F, device=dev)
        U = torch.zeros_like(F)
        for _ in range(warmup):
            U.zero_()
            b.solve(F, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            U.zero_()
            st = b.solve(F, U)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"setup_s": setup, "ms_per_solve": 1e3 * dt, "dofs_per_s": len(sig) * (n - 1) / dt,
                     "cycles_per_sigma": [x["cycles"] for x in st], "fallback": [x.get("fallback") for x in st],
                     "learned_setup_s": learned_s,
                     "max_div_norm": float(b.div_norm(U).max())}
        if sched:
            ms = b.time_kernel(1, 5, reps=50)
            z = b.sizes()
            alg = len(sig) * (4 * z["nnz"] + 3 * 4 * z["n"])
            out["fp32_residual_finest"] = {"ms": ms, "GBps": alg / (ms * 1e-3) / 1e9,
                                           "stored_values_per_problem": z["nnz"]}
        b.close()
    out["speedup_fp32_vs_fp64_additive"] = (out["fp64_additive_fixed_damping"]["ms_per_solve"] /
                                           out["fp32_refined_learned_chebyshev"]["ms_per_solve"])
    return out


def oseen_mlp_legs(dev, steps=3, warmup=1):
    """The learned-damping Oseen batch (context): 2D generalized Oseen, k=2,
    128^2, 6 grids, sigma = 1, nu in {1, 0.1, 0.01} x |a|h/nu in {0, 0.25,
    0.5, 1} (rotation), the twelve problems as one batch with the
    manufactured load, autotuned, from U = 0 to 1e-8: FP64 fixed damping
    V(2,2) against FP32 refinement with the network's constant dampings and
    steps, and with its Chebyshev schedule."""
    import torch
    import workloads
    from paper_1705_09282_amd.dfmg import BatchSolver
    from paper_1705_09282_amd import learned
    probs = [workloads.oseen2d(nu, peh) for nu in workloads.OSEEN2D_NUS for peh in workloads.OSEEN2D_PEH]
    p0 = probs[0]
    out = {"workload": "2D generalized Oseen, k=2, 128^2, 6 grids, sigma=1, nu in {1, 0.1, 0.01} x |a|h/nu in "
                       "{0, 0.25, 0.5, 1} (rotation), 12 problems as one batch, manufactured load, tol 1e-8, U0=0"}
    for name, prec, mode in (("fp64_fixed_damping", 0, None), ("fp32_refined_learned_constant_damping", 1, "constant"),
                             ("fp32_refined_learned_chebyshev", 1, "chebyshev")):
        b = BatchSolver(2, p0["N"], p0["L"], p0["k"], [p["nu"] for p in probs], [p["sigma"] for p in probs],
                        [p["c"] for p in probs], precision=prec, max_cycles=200).bind(dev)
        b.autotune(reps=10)
        if mode == "constant":
            learned.apply(b)
        elif mode == "chebyshev":
            learned.apply_chebyshev(b)
        F = torch.tensor(b.manufactured_rhs(), device=dev)
        U = torch.zeros_like(F)
        for _ in range(warmup):
            U.zero_()
            b.solve(F, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            U.zero_()
            st = b.solve(F, U)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"ms_per_solve": 1e3 * dt, "dofs_per_s": len(probs) * (b.n - 1) / dt,
                     "cycles": [x["cycles"] for x in st], "fallbacks": int(sum(x["fallback"] for x in st)),
                     "steps_per_level_finest_first": b.get_smoothing()[0],
                     "max_div_norm": float(b.div_norm(U).max())}
        b.close()
    base = out["fp64_fixed_damping"]["ms_per_solve"]
    out["speedup_constant_damping"] = base / out["fp32_refined_learned_constant_damping"]["ms_per_solve"]
    out["speedup_chebyshev"] = base / out["fp32_refined_learned_chebyshev"]["ms_per_solve"]
    return out


def mixed_batch_legs(dev, steps=3, warmup=1):
    """The mixed batch (context): 256 independent 2D problems of the seeded
    mix (grids 32^2..128^2, k in {1, 2}, sigma log-uniform in [1e-2, 1e4],
    nu = 1, rotation |a| in [0, 10]), one captured graph with a branch per
    mesh group, kernels and tiles autotuned per group; the manufactured load,
    solved from U = 0 to 1e-8: FP64 with the fixed damping V(2,2) against
    FP32 refinement with the learned Chebyshev schedule."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_09282_amd.dfmg import MultiSolver
    from paper_1705_09282_amd import learned
    probs = workloads.batch2d()
    meshes = [(p["d"], p["N"], p["L"], p["k"]) for p in probs]
    out = {"workload": f"{len(probs)} independent 2D generalized Stokes/Oseen problems, grids 32^2..128^2, "
                       "k in {1,2}, sigma log-uniform [1e-2,1e4], nu=1, |a| in [0,10] (seed 5), coarsest 4x4, "
                       "manufactured load, tol 1e-8, U0=0"}
    for name, prec, sched in (("fp64_fixed_damping", 0, False), ("fp32_refined_learned_chebyshev", 1, True)):
        t0 = time.perf_counter()
        m = MultiSolver(meshes, [p["nu"] for p in probs], [p["sigma"] for p in probs], [p["c"] for p in probs],
                        precision=prec).bind(dev)
        m.autotune()
        if sched:
            learned.apply_chebyshev(m)
        setup = time.perf_counter() - t0
        F = torch.tensor(m.manufactured_rhs(), device=dev)
        U = torch.zeros_like(F)
        for _ in range(warmup):
            U.zero_()
            m.solve(F, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            U.zero_()
            st = m.solve(F, U)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        cyc = [x["cycles"] for x in st]
        out[name] = {"setup_and_tuning_s": setup, "ms_per_solve": 1e3 * dt,
                     "dofs_per_s": (m.n_total - len(probs)) / dt, "mesh_groups": m.n_groups,
                     "cycles_mean": float(np.mean(cyc)), "cycles_max": int(max(cyc)),
                     "fallbacks": int(sum(bool(x.get("fallback")) for x in st)),
                     "max_div_norm": float(m.div_norm(U).max())}
        m.close()
    out["speedup_fp32_learned_vs_fp64_fixed"] = (out["fp64_fixed_damping"]["ms_per_solve"] /
                                                out["fp32_refined_learned_chebyshev"]["ms_per_solve"])
    return out


def cnab_legs(dev, nsteps=10):
    """Navier-Stokes by Crank-Nicolson / Adams-Bashforth steps (context):
    2D, k=2, 256^2, 6 grids, nu = 0.1, dt = 1e-3 (sigma = 2000; |u| dt / h
    stays below 1 for the explicit convection), driven from rest by the
    steady Stokes forcing f = -nu Lap u + grad p of the manufactured
    solution (load of 2 f); each step solves its generalized Stokes problem
    to 1e-8 from the previous velocity.  Plain FP64 (fixed damping V(2,2))
    against FP32 refinement with the learned Chebyshev schedule; nsteps
    timed steps after one untimed."""
    import torch
    from paper_1705_09282_amd.dfmg import Solver
    from paper_1705_09282_amd import learned
    nu, dt = 0.1, 1e-3
    out = {"workload": "Navier-Stokes, CN/AB steps (equation GS), 2D k=2 256^2, 6 grids, nu=0.1, dt=1e-3, "
                       "steady Stokes forcing of the manufactured solution, from rest, tol 1e-8 per step"}
    steady = Solver(2, 256, 6, 2, nu=nu, sigma=0.0)
    f2 = 2.0 * steady.manufactured_rhs()  # load of 2 f, f = -nu Lap u + grad p
    steady.close()
    for name, prec, lrn in (("fp64_fixed_damping", 0, False), ("fp32_refined_learned_chebyshev", 1, True)):
        s = Solver(2, 256, 6, 2, nu=nu, sigma=2.0 / dt, precision=prec, time_stepping=1).bind(dev)
        s.autotune(reps=10)
        if lrn:
            learned.apply_chebyshev(s)
        F2 = torch.tensor(f2, device=dev)
        prev, U = None, torch.zeros_like(F2)
        cyc = []
        for i in range(nsteps + 1):
            if i == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            Un = torch.empty_like(U)
            st = s.cnab_step(F2, prev, U, Un)
            prev, U = U, Un
            if i >= 1:
                cyc.append(st[0]["cycles"])
        torch.cuda.synchronize()
        dt_step = (time.perf_counter() - t0) / nsteps
        out[name] = {"ms_per_step": 1e3 * dt_step, "dofs_per_s": (s.n - 1) / dt_step, "cycles_per_step": cyc,
                     "div_norm_last": s.div_norm(U), "velocity_l2_coef_last": float(torch.linalg.norm(U))}
        s.close()
    out["speedup"] = out["fp64_fixed_damping"]["ms_per_step"] / out["fp32_refined_learned_chebyshev"]["ms_per_step"]
    return out


def guermond_legs(dev, nsteps=3):
    """Navier-Stokes by Guermond's semi-implicit steps (context): the same
    flow as the CN/AB leg (2D, k=2, 256^2, 6 grids, nu = 0.1, dt = 1e-3,
    steady Stokes forcing, from rest), each step a generalized Oseen problem
    advected by 3/2 u^n - 1/2 u^{n-1} (u^0 at the first step), solved to
    1e-8 with fixed damping V(2,2).  The operator changes every step, so
    each step builds a new context on the host (setup seconds, reported
    apart) before its load kernel and solve (GPU milliseconds)."""
    import torch
    from paper_1705_09282_amd.dfmg import Solver
    nu, dt = 0.1, 1e-3
    nv = 2 * (256 + 1) * (256 + 2)
    out = {"workload": "Navier-Stokes, Guermond steps (equation GO), 2D k=2 256^2, 6 grids, nu=0.1, dt=1e-3, "
                       "steady Stokes forcing of the manufactured solution, from rest, tol 1e-8 per step"}
    steady = Solver(2, 256, 6, 2, nu=nu, sigma=0.0)
    F2 = torch.tensor(2.0 * steady.manufactured_rhs(), device=dev)
    steady.close()
    for name, prec in (("fp64_fixed_damping", 0), ("fp32_refined_fixed_damping", 1)):
        prev, U = None, torch.zeros_like(F2)
        setup, solve, cyc = [], [], []
        for i in range(nsteps):
            a = U[:nv] if prev is None else 1.5 * U[:nv] - 0.5 * prev[:nv]
            t0 = time.perf_counter()
            s = Solver(2, 256, 6, 2, nu=nu, sigma=2.0 / dt, c=1.0, adv_kind=3, adv_coeffs=a.cpu().numpy(),
                       precision=prec, time_stepping=1).bind(dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Fd = torch.empty_like(F2)
            s.go_rhs(F2, U, Fd)
            Un = U.clone()
            st = s.solve(Fd, Un)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            setup.append(t1 - t0)
            solve.append(1e3 * (t2 - t1))
            cyc.append(st["cycles"])
            prev, U = U, Un
            div = s.div_norm(U)
            s.close()
        out[name] = {"setup_s_per_step": setup, "gpu_ms_per_step": solve, "cycles_per_step": cyc,
                     "div_norm_last": div}
    return out


def roofline_hbm(dev, reps=50):
    """The FP32 residual on an operator that cannot stay in the 256 MB
    Infinity Cache: one problem of the same workload on 1024^2 elements
    (8 grids; its FP32 values take 0.8 GB), timed with HIP events on the
    library stream over `reps` launches."""
    from paper_1705_09282_amd.dfmg import Solver
    t0 = time.perf_counter()
    s = Solver(2, 1024, 8, 2, precision=1).bind(dev)
    setup = time.perf_counter() - t0
    ms = s.time_kernel(1, 7, reps=reps)
    z = s.sizes()
    alg = 4 * z["nnz"] + 3 * 4 * z["n"]
    achieved = alg / (ms * 1e-3) / 1e9
    s.close()
    return {"bound": "hbm", "kernel": "k_spmv<2,2,1,true,false,false,float,true> (FP32 residual, one problem of "
                                      "1024x1024 elements, k=2; 0.8 GB of values, streamed with non-temporal loads)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic({"n_elem": 1024, "levels": 8, "problems": 1}, TRAFFIC_FILE_HBM),
            "alg_bytes_per_launch": alg, "avg_launch_ms": ms, "setup_s": setup}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-elem", type=int, default=256)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="also run a plain device copy of MB megabytes (reference for HBM byte counters)")
    ap.add_argument("--tuning-cache", default=None, metavar="JSON",
                    help="reuse the kernel variants stored in JSON by an earlier run (a profiled run then times "
                         "the variants the unprofiled run chose); stores them when absent")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the timed path's batch, one solve, then the dominant kernel's timing loop and "
                         "200 finest-grid smoothing steps (for profiler and counter runs)")
    ap.add_argument("--roofline-hbm-only", action="store_true",
                    help="only the HBM-resident residual leg (1024^2, one problem)")
    ap.add_argument("--no-hbm-leg", action="store_true", help="skip the HBM-resident residual leg")
    ap.add_argument("--no-paper-legs", action="store_true", help="skip the paper's Oseen problems (context legs)")
    ap.add_argument("--only", choices=("timed", "multiplicative", "mixed"), default=None,
                    help="build and time one path only (for kernel traces): the timed path, the multiplicative "
                         "FP64 V(1,2) batch, or the mixed 256-problem batch with FP32 refinement and the learned "
                         "schedule; prints its ms per step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver runs each problem on a "
              f"single device and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {3} copies of {n * 8} bytes", file=sys.stderr, flush=True)
        del src, dst
    from paper_1705_09282_amd.dfmg import BatchSolver
    sigmas = list(workloads.STOKES2D_SIGMAS)
    cfg = workloads.stokes2d(1.0, N=args.n_elem, L=args.levels)

    from paper_1705_09282_amd import learned
    models = {"constant": learned.load(), "chebyshev": learned.load(learned.CHEB_WEIGHTS)}

    def make_batch(precision, use_learned=None, **opts):
        b = BatchSolver(cfg["d"], cfg["N"], cfg["L"], cfg["k"], [cfg["nu"]] * len(sigmas), sigmas,
                        precision=precision, **opts).bind(dev)
        tag = "-mult" if opts.get("multiplicative") else ""
        tuning = b.autotune(reps=20, cache=args.tuning_cache,
                            key=f"{cfg['N']}-{cfg['L']}-{precision}-{use_learned or 'fixed'}{tag}")
        if use_learned:
            t0 = time.perf_counter()
            learned.apply(b, models[use_learned])
            # the schedule's eigenvalue estimates (30 power iterations per
            # level and problem, host norms) are made here
            tuning["learned_setup_s"] = time.perf_counter() - t0
        print(f"[bench] batch ready: precision {precision}, {use_learned or 'fixed damping'}{tag}", file=sys.stderr,
              flush=True)
        F = torch.tensor(b.manufactured_rhs(), device=dev)
        U = torch.zeros_like(F)
        return b, F, U, tuning

    def run(b, F, U):
        """warm-up, then the timed steps; returns (seconds, stats of the last step)"""
        def step():
            U.zero_()
            return b.solve(F, U, tol=args.tol)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            stats = step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, stats

    def roofline(b, F, U):
        """dominant kernel of the timed path: the finest-grid FP32 residual of
        the whole batch, timed with HIP events on the library stream in the
        launch configuration of the cycles"""
        ms = b.time_kernel(1, args.levels - 1, reps=200)
        z = b.sizes()
        alg = len(sigmas) * (4 * z["nnz"] + 3 * 4 * z["n"])
        achieved = alg / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": "k_spmv<2,2,1,true,false,false,float,false> (finest-grid FP32 residual r = F - K U, "
                                          f"{len(sigmas)} problems per launch)",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic({"n_elem": args.n_elem, "levels": args.levels}),
                "alg_bytes_per_launch": alg,
                "avg_launch_ms": ms}

    if args.roofline_hbm_only:
        print(json.dumps({"roofline_hbm": roofline_hbm(dev, reps=200)}), flush=True)
        return

    if args.only == "mixed":
        from paper_1705_09282_amd.dfmg import MultiSolver
        probs = workloads.batch2d()
        m = MultiSolver([(p["d"], p["N"], p["L"], p["k"]) for p in probs], [p["nu"] for p in probs],
                        [p["sigma"] for p in probs], [p["c"] for p in probs], precision=1).bind(dev)
        m.autotune()
        learned.apply_chebyshev(m)
        F = torch.tensor(m.manufactured_rhs(), device=dev)
        U = torch.zeros_like(F)
        T, st = run(m, F, U)
        print(json.dumps({"path": "mixed", "ms_per_step": 1e3 * T / args.steps, "mesh_groups": m.n_groups,
                          "cycles_max": max(x["cycles"] for x in st), "steps": args.steps,
                          "warmup": args.warmup}), flush=True)
        m.close()
        return

    if args.only:
        if args.only == "timed":
            b, F, U, tun = make_batch(1, use_learned="chebyshev")
        else:
            b, F, U, tun = make_batch(0, multiplicative=1, nu1=1, nu2=2)
        T, st = run(b, F, U)
        print(json.dumps({"path": args.only, "ms_per_step": 1e3 * T / args.steps,
                          "cycles_per_sigma": [x["cycles"] for x in st], "steps": args.steps, "warmup": args.warmup,
                          "tuning": {k: v for k, v in tun.items() if k != "ms"},
                          "steps_per_level_finest_first": b.get_smoothing()[0]}), flush=True)
        b.close()
        return

    if args.roofline_only:
        # the residual's roofline, then 200 finest-grid smoothing steps of the
        # same batch (the local solves and the per-DOF update, for counter runs)
        b32, F32, U32, _ = make_batch(1, use_learned="chebyshev")
        U32.zero_()
        b32.solve(F32, U32, tol=args.tol)
        out = {"roofline": roofline(b32, F32, U32)}
        out["fp32_smoothing_step_ms"] = b32.time_kernel(3, args.levels - 1, reps=200)
        print(json.dumps(out), flush=True)
        b32.close()
        return

    t_setup = time.perf_counter()
    b64, F64, U64, tun64 = make_batch(0)
    bfx, Ffx, Ufx, tunfx = make_batch(1)
    blc, Flc, Ulc, _ = make_batch(1, use_learned="constant")
    bc64, Fc64, Uc64, _ = make_batch(0, use_learned="chebyshev")
    b32, F32, U32, tun32 = make_batch(1, use_learned="chebyshev")
    setup_s = time.perf_counter() - t_setup
    bm, Fm, Um, _ = make_batch(0, multiplicative=1, nu1=1, nu2=2)
    z = b64.sizes()
    dofs = len(sigmas) * (z["n"] - 1)
    print(f"[bench] setup of 5 batches of {len(sigmas)} problems: {setup_s:.1f} s, DOFs/step {dofs}",
          file=sys.stderr, flush=True)

    T64, stats64 = run(b64, F64, U64)
    print(f"[bench] plain FP64 batch: {args.steps} steps in {T64:.3f} s", file=sys.stderr, flush=True)
    Tfx, statsfx = run(bfx, Ffx, Ufx)
    print(f"[bench] FP32-refined batch, fixed damping: {args.steps} steps in {Tfx:.3f} s", file=sys.stderr,
          flush=True)
    Tlc, statslc = run(blc, Flc, Ulc)
    print(f"[bench] FP32-refined batch, learned constant damping: {args.steps} steps in {Tlc:.3f} s",
          file=sys.stderr, flush=True)
    Tc64, statsc64 = run(bc64, Fc64, Uc64)
    print(f"[bench] FP64 batch, learned Chebyshev schedule: {args.steps} steps in {Tc64:.3f} s", file=sys.stderr,
          flush=True)
    Tm, statsm = run(bm, Fm, Um)
    print(f"[bench] FP64 batch, multiplicative Schwarz V(1,2): {args.steps} steps in {Tm:.3f} s", file=sys.stderr,
          flush=True)
    T, stats = run(b32, F32, U32)
    print(f"[bench] learned Chebyshev schedule + FP32-refined batch: {args.steps} steps in {T:.3f} s",
          file=sys.stderr, flush=True)

    n = z["n"]
    nv = z["n_vel"]
    errs = []
    for p in range(len(sigmas)):
        a = U32[p * n:p * n + nv]
        ref = U64[p * n:p * n + nv]
        errs.append(float(torch.linalg.norm(a - ref) / torch.linalg.norm(ref)))
    cycles = [st["cycles"] for st in stats]
    divs = [float(x) for x in b32.div_norm(U32)]
    value = args.steps * dofs / T
    value64 = args.steps * dofs / T64
    tuning = tun32

    rl = roofline(b32, F32, U32)
    # context: the FP64 residual and the smoothing steps of the finest grid
    z = b64.sizes()
    ms64 = b64.time_kernel(0, args.levels - 1, reps=100)
    gbs64 = len(sigmas) * (8 * z["nnz"] + 3 * 8 * z["n"]) / (ms64 * 1e-3) / 1e9
    sm64 = b64.time_kernel(2, args.levels - 1, reps=50)
    sm32 = b32.time_kernel(3, args.levels - 1, reps=50)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"stokes2d: 2D generalized Stokes, k=2, {args.n_elem}x{args.n_elem} elements, "
                        f"{args.levels} grids, nu=1, sigma in {{1e-2,1,1e2,1e4}}, additive Schwarz V-cycles, "
                        f"tol {args.tol:g}, U0=0",
            "path": "batched: learned Chebyshev damping schedule (network: interval ratio and smoothing steps per "
                    "level), FP32 V-cycles in FP64 iterative refinement, 4 problems per launch (plain_fp64: "
                    "fixed damping, V(2,2))",
            "steps_per_level_finest_first": b32.get_smoothing()[0],
            "alpha_per_sigma": [[round(x, 3) for x in row] for row in b32.get_alpha().tolist()],
            "lmax_per_sigma": [[round(x, 4) for x in row] for row in b32.get_lmax().tolist()],
            "finest_pre_smoothing_dampings_sigma1": [round(x, 4) for x in
                                                     b32.get_schedule()[1, 0, 0, :b32.get_smoothing()[0][0]]],
            "fallback_per_sigma": [st["fallback"] for st in stats],
            "dofs_per_step": dofs,
            "cycles_per_sigma": cycles,
            "vcycles_per_s": args.steps * sum(cycles) / T,
            "div_norm_per_sigma": divs,
            "vel_rel_err_vs_plain_fp64_per_sigma": errs,
            "plain_fp64": {"value": value64, "ms_per_step": 1e3 * T64 / args.steps,
                           "cycles_per_sigma": [st["cycles"] for st in stats64],
                           "vcycles_per_s": args.steps * sum(st["cycles"] for st in stats64) / T64},
            "fp32_fixed_damping": {"value": args.steps * dofs / Tfx, "ms_per_step": 1e3 * Tfx / args.steps,
                                   "cycles_per_sigma": [st["cycles"] for st in statsfx]},
            "fp32_learned_constant_damping": {
                "value": args.steps * dofs / Tlc, "ms_per_step": 1e3 * Tlc / args.steps,
                "cycles_per_sigma": [st["cycles"] for st in statslc],
                "steps_per_level_finest_first": blc.get_smoothing()[0],
                "eta_per_sigma": [[round(x, 4) for x in row] for row in blc.get_eta().tolist()]},
            "fp64_learned_chebyshev": {"value": args.steps * dofs / Tc64, "ms_per_step": 1e3 * Tc64 / args.steps,
                                       "cycles_per_sigma": [st["cycles"] for st in statsc64]},
            "fp64_multiplicative_v12": {"value": args.steps * dofs / Tm, "ms_per_step": 1e3 * Tm / args.steps,
                                        "cycles_per_sigma": [st["cycles"] for st in statsm],
                                        "div_norm_per_sigma": [float(x) for x in bm.div_norm(Um)]},
            "speedup_vs_plain_fp64": value / value64,
            "setup_s": setup_s,
            "lmax_estimate_s": tuning.get("learned_setup_s"),
            "tuning": {"lpr": tuning["lpr"],
                       # the FP32 cycle of the refinement runs smoother form 3
                       # where tuned so and form 4 otherwise (level 0: exact)
                       "smoother_fp32_cycle": [None] + [3 if f == 3 else 4 for f in tuning["smoother"][1:]],
                       "smoother_fp64_residual_path": tuning["smoother"]},
            "finest_grid_kernels_ms": {"fp64_residual": ms64, "fp64_residual_GBps": gbs64,
                                       "fp64_smoothing_step": sm64, "fp32_smoothing_step": sm32},
        },
        "roofline": rl,
    }
    U32_sigma1 = U32[n:2 * n].cpu().numpy()
    for s in (b64, bfx, blc, bc64, b32, bm):
        s.close()
    del b64, bfx, blc, bc64, b32, bm, F64, U64, Ffx, Ufx, Flc, Ulc, Fc64, Uc64, F32, U32, Fm, Um
    torch.cuda.empty_cache()
    if not args.no_hbm_leg:
        print("[bench] HBM-resident residual leg (1024^2)", file=sys.stderr, flush=True)
        line["roofline_hbm"] = roofline_hbm(dev)
    if not args.no_paper_legs:
        print("[bench] the paper's Oseen problems (context)", file=sys.stderr, flush=True)
        line["config"]["paper_oseen_2d"] = paper_oseen_legs(dev)
        print("[bench] the 3D workload (context)", file=sys.stderr, flush=True)
        line["config"]["stokes3d"] = stokes3d_legs(dev)
        print("[bench] the learned-damping Oseen batch (context)", file=sys.stderr, flush=True)
        line["config"]["oseen_learned"] = oseen_mlp_legs(dev)
        print("[bench] the mixed 256-problem batch (context)", file=sys.stderr, flush=True)
        line["config"]["mixed_batch"] = mixed_batch_legs(dev)
        print("[bench] the quarter annulus (context)", file=sys.stderr, flush=True)
        line["config"]["annulus"] = annulus_legs(dev)
        print("[bench] Navier-Stokes CN/AB steps (context)", file=sys.stderr, flush=True)
        line["config"]["navier_stokes_cnab"] = cnab_legs(dev)
        print("[bench] Navier-Stokes Guermond steps (context)", file=sys.stderr, flush=True)
        line["config"]["navier_stokes_guermond"] = guermond_legs(dev)
    if not args.no_cpu_baseline and args.n_elem == 256 and args.levels == 6:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"], line["config"]["vel_rel_err_vs_oracle_sigma1"] = cpu_baseline(args.tol, U32_sigma1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
