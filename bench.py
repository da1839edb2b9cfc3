#!/usr/bin/env python3
"""Throughput of the divergence-conforming multigrid solver on one MI355X.

Workload (synthetic, seeded): 2D generalized Stokes on the unit square,
pressure degree k=2 (velocity S^{3,2} x S^{2,3}), 256x256 elements, 6 grids
(256 .. 8), nu = 1, sigma in {1e-2, 1, 1e2, 1e4}, load vector of the
manufactured solution u = curl(sin^2(pi x) sin^2(pi y)), p = sin(2 pi x)
sin(2 pi y).  One step solves all four problems from U = 0 to relative
residual 1e-8 with V(2,2) cycles; inputs are resident in HBM before timing.

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
KERNEL_SRC = os.path.join(ROOT, "paper_1705_09282_amd", "csrc", "spmv.hip")


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the finest residual kernel from the committed
    rocprofv3 counter runs, or None if missing or taken on other kernel code."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(tol):
    """The oracle as it stands, on one of the four problems (sigma = 1), one
    full solve to tol from U = 0; setup excluded as for the GPU."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    import workloads
    from oracle.multigrid import Hierarchy, solve
    from oracle.assemble import load_vector
    from oracle.manufactured import forcing
    cfg = workloads.stokes2d(1.0)
    with threadpool_limits(1):
        h = Hierarchy(cfg["d"], cfg["N"], cfg["k"], cfg["L"], cfg["nu"], cfg["sigma"])
        F = load_vector(h.finest.disc, forcing(cfg["d"], cfg["nu"], cfg["sigma"]))
        t0 = time.perf_counter()
        U, hist = solve(h, F, tol=tol)
        dt = time.perf_counter() - t0
    dofs = h.finest.disc.dofs()
    return {"value": dofs / dt, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": "sigma=1 problem only (1 of 4): one full FP64 oracle solve to 1e-8 from U=0, "
                      "256x256, k=2, 6 grids, V(2,2), setup excluded, BLAS limited to 1 thread",
            "seconds": dt, "cycles": len(hist) - 1}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver runs each problem on a "
              f"single device and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_1705_09282_amd.dfmg import Solver

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
    def make_problems(precision):
        probs = []
        for sigma in workloads.STOKES2D_SIGMAS:
            cfg = workloads.stokes2d(sigma, N=args.n_elem, L=args.levels)
            s = Solver(cfg["d"], cfg["N"], cfg["L"], cfg["k"], nu=cfg["nu"], sigma=cfg["sigma"],
                       precision=precision).bind(dev)
            tuning = s.autotune(reps=20)
            F = torch.tensor(s.manufactured_rhs(), device=dev)
            U = torch.zeros_like(F)
            probs.append((sigma, s, F, U, s.sizes(), tuning))
        return probs

    def run(probs):
        """warm-up, then the timed steps; returns (seconds, stats of the last step)"""
        def step():
            out = []
            for sigma, s, F, U, z, _ in probs:
                U.zero_()
                out.append(s.solve(F, U, tol=args.tol))
            return out
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            stats = step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, stats

    t_setup = time.perf_counter()
    plain = make_problems(0)
    mixed = make_problems(1)
    setup_s = time.perf_counter() - t_setup
    dofs = sum(z["n"] - 1 for *_, z, _ in plain)
    print(f"[bench] setup of 2x{len(plain)} problems: {setup_s:.1f} s, DOFs/step {dofs}", file=sys.stderr, flush=True)

    T64, stats64 = run(plain)
    print(f"[bench] plain FP64: {args.steps} steps in {T64:.3f} s", file=sys.stderr, flush=True)
    T, stats = run(mixed)
    print(f"[bench] FP32-refined: {args.steps} steps in {T:.3f} s", file=sys.stderr, flush=True)

    # error of the refined solutions against the plain FP64 solutions of the same step
    import numpy as np
    errs = []
    for (_, _, _, U64, z, _), (_, _, _, U32, _, _) in zip(plain, mixed):
        nv = z["n_vel"]
        a, b = U32[:nv].double(), U64[:nv].double()
        errs.append(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)))
    cycles = [st["cycles"] for st in stats]
    divs = [s.div_norm(U) for _, s, _, U, _, _ in mixed]
    value = args.steps * dofs / T
    value64 = args.steps * dofs / T64
    probs = plain
    tuning = plain[-1][5]

    # roofline of the dominant kernel: finest-grid residual of the sigma = 1 problem
    _, s1, F1, U1, z1, _ = probs[1]
    r = torch.empty_like(F1)
    ms = s1.time_residual(args.levels - 1, F1, U1, r, reps=200)
    alg_bytes = 8 * z1["nnz"] + 3 * 8 * z1["n"]
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    traffic = measured_traffic()

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
                        f"{args.levels} grids, nu=1, sigma in {{1e-2,1,1e2,1e4}}, V(2,2) additive Schwarz, "
                        f"tol {args.tol:g}, U0=0",
            "path": "FP32 V-cycles in FP64 iterative refinement (fixed damping)",
            "dofs_per_step": dofs,
            "cycles_per_sigma": cycles,
            "vcycles_per_s": args.steps * sum(cycles) / T,
            "div_norm_per_sigma": divs,
            "vel_rel_err_vs_plain_fp64_per_sigma": errs,
            "plain_fp64": {"value": value64, "ms_per_step": 1e3 * T64 / args.steps,
                           "cycles_per_sigma": [st["cycles"] for st in stats64],
                           "vcycles_per_s": args.steps * sum(st["cycles"] for st in stats64) / T64},
            "speedup_vs_plain_fp64": value / value64,
            "setup_s": setup_s,
            "tuning_last_problem": {"lpr": tuning["lpr"], "smoother": tuning["smoother"]},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_spmv<2,2> (finest-grid residual r = F - K U)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": ms,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.tol)
    for _, s, _, _, _, _ in plain + mixed:
        s.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
