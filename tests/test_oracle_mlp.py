"""Pins of the oracle's learned-damping network: gradient vs central finite
differences in FP64, masked loss, Adam against its closed form on a quadratic."""
import numpy as np

from oracle import mlp


def _data(n=13, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (n, mlp.NIN))
    Y = rng.uniform(-2, 2, (n, mlp.NOUT))
    M = (rng.uniform(0, 1, (n, mlp.NOUT)) > 0.2).astype(float)
    return X, Y, M


def test_gradient_matches_finite_differences():
    X, Y, M = _data()
    th = mlp.init(1) + 0.05 * np.random.default_rng(2).standard_normal(mlp.NPARAM)
    g = mlp.grad(th, X, Y, M)
    rng = np.random.default_rng(3)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = eps
        fd = (mlp.loss(th + e, X, Y, M) - mlp.loss(th - e, X, Y, M)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd)


def test_masked_loss_and_shapes():
    X, Y, M = _data()
    th = mlp.init(4)
    Z = mlp.forward(th, X)
    assert Z.shape == (13, mlp.NOUT) and mlp.NPARAM == 1546
    M0 = np.zeros_like(M)
    M0[0, 0] = 1.0
    np.testing.assert_allclose(mlp.loss(th, X, Y, M0), (Z[0, 0] - Y[0, 0]) ** 2)


def test_adam_on_quadratic():
    """Adam's first step moves every coordinate by lr * sign(g) (bias-corrected)."""
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 2.0])
    new, m, v = mlp.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    np.testing.assert_allclose(new, th - 0.1 * np.sign(g), rtol=1e-6)


def test_step_rounding():
    np.testing.assert_array_equal(mlp.steps(np.array([-3.0, 0.4, 1.5, 2.49, 2.5, 7.6, 20.0])), [1, 1, 2, 2, 3, 8, 8])
