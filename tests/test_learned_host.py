"""Host logic of the learned parts that runs without a GPU: the fallback
thresholds (nearest training points on the unit square and cube, measured on
the problem itself on mapped domains) and the network inputs of a solver."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1705_09282_amd import learned


def fake_solver(geometry=0, nus=(1.0, 0.1), sigmas=(1.0, 100.0), cs=(0.0, 0.0), dim=2):
    return SimpleNamespace(geometry=geometry, adv_kind=None, nus=list(nus), sigmas=list(sigmas), cs=list(cs),
                           n_elem=64, k=2, dim=dim)


def test_rho_plain_for_takes_the_largest_of_the_nearest():
    X = np.array([[0.0, 0.0, 0.0, 0.5], [0.0, 0.1, 0.0, 0.5], [1.0, 1.0, 0.0, 0.5], [0.0, 0.05, 0.0, -0.5]])
    model = {"train": {"X": X, "worst_plain": np.array([0.3, 0.4, 0.9, 0.6])}}
    got = learned.rho_plain_for(model, [[0.0, 0.02, 0.0, 0.5]], neighbours=2)
    assert got.tolist() == [0.4]  # rows 0 and 1 are nearest; row 2 (0.9) is far
    got = learned.rho_plain_for(model, [[0.0, 0.02, 0.0, 0.5]], neighbours=3)
    assert got.tolist() == [0.6]


def test_problem_features_follow_the_network_inputs():
    s = fake_solver(nus=(1.0, 0.01), sigmas=(1e-2, 1e4), cs=(0.0, 2.0 * math.sqrt(2.0)))
    F = learned.problem_features(s)
    assert F.shape == (2, 4)
    np.testing.assert_allclose(F[0], [0.0, -0.5, 0.0, 0.5])
    # |a| = c / sqrt(2) for the rotation, h = 1 / 64, nu = 0.01: |a| h / nu = 2 / 64 / 0.01
    np.testing.assert_allclose(F[1], [-1.0, 1.0, 2.0 / 64 / 0.01, 0.5])


def test_fallback_thresholds_square_uses_training_points(monkeypatch):
    model = learned.load(learned.CHEB_WEIGHTS)
    s = fake_solver()
    monkeypatch.setattr(learned, "measured_worst_plain", lambda solver: pytest.fail("must not measure"))
    got = learned.fallback_thresholds(model, s)
    np.testing.assert_array_equal(got, learned.rho_plain_for(model, learned.problem_features(s)))
    assert ((got > 0) & (got < 1)).all()


@pytest.mark.parametrize("geometry,dim", [(1, 2), (1, 3), (0, 3)])
def test_fallback_thresholds_mapped_or_3d_is_measured(monkeypatch, geometry, dim):
    model = learned.load(learned.CHEB_WEIGHTS)
    s = fake_solver(geometry=geometry, dim=dim)
    calls = []

    def measured(solver):
        calls.append(solver)
        return np.array([0.93, 0.94])

    monkeypatch.setattr(learned, "measured_worst_plain", measured)
    got = learned.fallback_thresholds(model, s)
    assert calls == [s]
    assert got.tolist() == [0.93, 0.94]
