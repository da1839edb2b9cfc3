"""The allocation-free gradient entry point (dfmg_mlp_grad_noalloc) through
the C-ABI against dfmg_mlp_grad on the same inputs: equal bit for bit (same
kernels, same summation order), on two calls in a row with the second on
fewer samples (the static scratch keeps the first call's rows, which the
second must not read), the largest allowed batch, and the size check."""
import numpy as np
import pytest

from oracle import mlp as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, (n, om.NIN)).astype(np.float32)
    Y = rng.normal(0.0, 1.0, (n, om.NOUT)).astype(np.float32)
    M = (rng.uniform(size=(n, om.NOUT)) < 0.8).astype(np.float32)
    W = (om.init(seed) + rng.normal(0.0, 0.1, om.NPARAM)).astype(np.float32)
    return [torch.tensor(a.ravel(), device="cuda") for a in (W, X, Y, M)]


def _both(n, seed):
    from paper_1705_09282_amd.dfmg import mlp_grad, mlp_grad_noalloc, MLP_NPARAM
    W, X, Y, M = _data(n, seed)
    out = []
    for noalloc in (False, True):
        G = torch.full((MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        if noalloc:
            mlp_grad_noalloc(W, X, Y, M, 0.01, G, loss)
        else:
            work = torch.zeros(n * (MLP_NPARAM + 1), dtype=torch.float32, device="cuda")
            mlp_grad(W, X, Y, M, 0.01, work, G, loss)
        torch.cuda.synchronize()
        out.append(np.concatenate([G.cpu().numpy(), loss.cpu().numpy()]))
    return out


def test_noalloc_grad_equals_grad():
    from paper_1705_09282_amd.dfmg import MLP_SCRATCH_SAMPLES
    for n, seed in ((300, 1), (37, 2), (MLP_SCRATCH_SAMPLES, 3), (1, 4)):
        print(f"\n[case] mlp_grad_noalloc n={n} seed={seed}", flush=True)
        a, b = _both(n, seed)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), (n, np.max(np.abs(a - b)))


def test_noalloc_grad_rejects_too_many_samples():
    from paper_1705_09282_amd.dfmg import mlp_grad_noalloc, MLP_NPARAM, MLP_SCRATCH_SAMPLES, DfmgError
    n = MLP_SCRATCH_SAMPLES + 1
    W, X, Y, M = _data(n, 5)
    G = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(DfmgError) as e:
        mlp_grad_noalloc(W, X, Y, M, 0.01, G, loss)
    assert e.value.code == -1
    assert torch.count_nonzero(G).item() == 0
