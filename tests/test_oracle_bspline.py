"""Pins of the oracle's B-spline layer against textbook facts."""
import numpy as np
import pytest

from oracle.bspline import open_knots, basis, basis_deriv, gauss_rule


@pytest.mark.parametrize("N", [1, 3, 8])
@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_partition_of_unity_and_count(N, q):
    kn = open_knots(N, q)
    assert len(kn) == N + 2 * q + 1
    x = np.concatenate([np.random.default_rng(1).uniform(0, 1, 50), [0.0, 1.0]])
    B = basis(kn, q, x)
    assert B.shape == (x.size, N + q)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert (B >= -1e-15).all()


@pytest.mark.parametrize("q", [1, 2, 3])
def test_derivative_matches_finite_difference(q):
    kn = open_knots(6, q)
    x = np.random.default_rng(2).uniform(0.01, 0.99, 40)
    # keep away from knots where derivatives of low degree jump
    x = x[np.min(np.abs(x[:, None] - np.arange(7)[None, :] / 6), axis=1) > 1e-3]
    eps = 1e-6
    fd = (basis(kn, q, x + eps) - basis(kn, q, x - eps)) / (2 * eps)
    np.testing.assert_allclose(basis_deriv(kn, q, x), fd, atol=2e-6 * 6 ** q)


def test_uniform_cardinal_values():
    """Uniform quadratic B-spline: 1/8, 3/4, 1/8 at element midpoints; cubic:
    1/6, 2/3, 1/6 at knots (textbook cardinal B-spline values)."""
    kn = open_knots(10, 2)
    # interior function 4 has support [2/10, 5/10]
    B = basis(kn, 2, np.array([0.25, 0.35, 0.45]))[:, 4]
    np.testing.assert_allclose(B, [1 / 8, 3 / 4, 1 / 8], atol=1e-15)
    kn = open_knots(10, 3)
    B = basis(kn, 3, np.array([0.3, 0.4, 0.5]))[:, 6]  # support [3/10, 7/10]
    np.testing.assert_allclose(B, [0.0, 1 / 6, 2 / 3], atol=1e-15)


def test_gauss_rule_integrates_polynomials():
    x, w = gauss_rule(5, 4)
    for p in range(8):
        np.testing.assert_allclose(np.sum(w * x ** p), 1.0 / (p + 1), rtol=1e-13)
