"""Batches of problems on different meshes (dfmg_multi_*): every problem's
solve equals the single-mesh batch of its group bit for bit (the same kernels
run on the same data, only on another stream and inside one graph), and the
small problems match the FP64 oracle; then the 256-problem mixed workload."""
import math

import numpy as np
import pytest

import workloads
from oracle.multigrid import Hierarchy, solve as oracle_solve
from oracle.assemble import load_vector, rotation_field
from oracle.manufactured import forcing

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIX = [((2, 16, 3, 1), 1.0, 1.0, 0.0), ((2, 32, 4, 2), 1.0, 1e2, 4.0), ((2, 16, 3, 1), 1.0, 1e-2, 2.0),
       ((2, 32, 4, 2), 1.0, 1.0, 0.0), ((2, 32, 4, 1), 1.0, 1e3, 8.0), ((2, 16, 3, 1), 0.5, 10.0, 0.0)]


def build_multi(mix, **opt):
    from paper_1705_09282_amd.dfmg import MultiSolver
    return MultiSolver([m for m, *_ in mix], [x[1] for x in mix], [x[2] for x in mix], [x[3] for x in mix],
                       **opt).bind()


@pytest.mark.parametrize("precision,use_graph", [(0, 1), (0, 0), (1, 1)])
def test_multi_equals_group_batches(precision, use_graph):
    from paper_1705_09282_amd.dfmg import BatchSolver
    print(f"\n[case] precision={precision} use_graph={use_graph}", flush=True)
    M = build_multi(MIX, precision=precision, use_graph=use_graph)
    assert M.n_groups == 3
    F = torch.tensor(M.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    st = M.solve(F, U, tol=1e-8)
    Uh = U.cpu().numpy()
    off = M.offsets
    for mesh in sorted(set(m for m, *_ in MIX)):
        idx = [i for i, x in enumerate(MIX) if x[0] == mesh]
        d, N, L, k = mesh
        B = BatchSolver(d, N, L, k, [MIX[i][1] for i in idx], [MIX[i][2] for i in idx], [MIX[i][3] for i in idx],
                        precision=precision, use_graph=use_graph).bind()
        Fb = torch.tensor(B.manufactured_rhs(), device="cuda")
        Ub = torch.zeros_like(Fb)
        sb = B.solve(Fb, Ub, tol=1e-8)
        Ubh = Ub.cpu().numpy()
        for j, i in enumerate(idx):
            assert np.array_equal(Fb.cpu().numpy()[j * B.n:(j + 1) * B.n], F.cpu().numpy()[off[i]:off[i + 1]])
            assert np.array_equal(Ubh[j * B.n:(j + 1) * B.n], Uh[off[i]:off[i + 1]]), (mesh, i)
            assert sb[j]["cycles"] == st[i]["cycles"] and sb[j]["history"] == st[i]["history"]
        B.close()
    res = M.residual_norm(F, U)
    div = M.div_norm(U)
    for i in range(len(MIX)):
        assert st[i]["converged"]
        assert res[i] <= 1e-8 * st[i]["fnorm"] * 1.0001
        assert div[i] < 1e-10
    M.close()


def test_multi_matches_oracle():
    M = build_multi(MIX[:3])
    F = torch.tensor(M.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    st = M.solve(F, U, tol=1e-8)
    Uh = U.cpu().numpy()
    for i, ((d, N, L, k), nu, sigma, c) in enumerate(MIX[:3]):
        adv = rotation_field(c) if c else None
        h = Hierarchy(d, N, k, L, nu, sigma, adv)
        Fo = load_vector(h.finest.disc, forcing(d, nu, sigma, adv))
        Uo, hist = oracle_solve(h, Fo, tol=1e-8)
        got = Uh[M.offsets[i]:M.offsets[i + 1]]
        nv = h.finest.disc.n_v
        err = np.linalg.norm(got[:nv] - Uo[:nv]) / np.linalg.norm(Uo[:nv])
        print(f"[oracle] problem {i} cycles {st[i]['cycles']} / {len(hist) - 1} vel err {err:.2e}", flush=True)
        assert st[i]["cycles"] == len(hist) - 1
        assert err < 1e-10
    M.close()


def test_multi_errors():
    from paper_1705_09282_amd.dfmg import MultiSolver, DfmgError
    with pytest.raises(DfmgError):  # multiplicative Schwarz runs in FP64 cycles only
        MultiSolver([(3, 8, 2, 1), (2, 16, 3, 1)], [1.0, 1.0], [1.0, 1.0], precision=1, multiplicative=1)
    with pytest.raises(DfmgError):
        MultiSolver([(2, 12, 4, 1)], [1.0], [1.0])  # 12 not divisible by 2^3
    M = MultiSolver([(2, 16, 3, 1)], [1.0], [1.0])
    F = torch.zeros(M.n_total, dtype=torch.float64, device="cuda")
    with pytest.raises(DfmgError):
        M.solve(F, F.clone())  # not bound
    M.close()


def test_mixed_batch_workload():
    """The 256-problem mixed workload (grids 32^2..128^2, k 1 and 2, sigma
    log-uniform, rotation |a| up to 10) in FP32 V-cycles inside FP64
    refinement: every problem converges to 1e-8 and stays divergence-free;
    two problems per group are compared with their single-mesh batch."""
    from paper_1705_09282_amd.dfmg import MultiSolver, BatchSolver
    probs = workloads.batch2d()
    meshes = [(p["d"], p["N"], p["L"], p["k"]) for p in probs]
    M = MultiSolver(meshes, [p["nu"] for p in probs], [p["sigma"] for p in probs], [p["c"] for p in probs],
                    precision=1).bind()
    print(f"\n[case] 256 problems, {M.n_groups} groups, {M.n_total} DOFs", flush=True)
    F = torch.tensor(M.manufactured_rhs(), device="cuda")
    U = torch.zeros_like(F)
    st = M.solve(F, U, tol=1e-8)
    div = M.div_norm(U)
    res = M.residual_norm(F, U)
    cyc = [s["cycles"] for s in st]
    print(f"[batch] cycles min {min(cyc)} max {max(cyc)} mean {np.mean(cyc):.1f}; max div {div.max():.1e}",
          flush=True)
    for i, s in enumerate(st):
        assert s["converged"], i
        assert res[i] <= 1e-8 * s["fnorm"] * 1.0001
    assert div.max() < 1e-10
    Uh = U.cpu().numpy()
    for mesh in sorted(set(meshes)):
        idx = [i for i, m in enumerate(meshes) if m == mesh][:2]
        d, N, L, k = mesh
        B = BatchSolver(d, N, L, k, [probs[i]["nu"] for i in idx], [probs[i]["sigma"] for i in idx],
                        [probs[i]["c"] for i in idx], precision=1).bind()
        Fb = torch.tensor(B.manufactured_rhs(), device="cuda")
        Ub = torch.zeros_like(Fb)
        sb = B.solve(Fb, Ub, tol=1e-8)
        for j, i in enumerate(idx):
            got = Uh[M.offsets[i]:M.offsets[i + 1]]
            ref = Ub.cpu().numpy()[j * B.n:(j + 1) * B.n]
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            # different batch sizes may pick different residual-kernel variants
            # (summation order), so agreement is to the solve tolerance
            assert err < 1e-6 and abs(sb[j]["cycles"] - st[i]["cycles"]) <= 1, (mesh, i, err)
        B.close()
    M.close()
