"""Pins of the misfit ERR of Eq. (eqerr) (Section 2) by its exact
identities."""
import numpy as np
import pytest

from oracle import misfit


@pytest.fixture
def obs():
    return np.random.default_rng(0).standard_normal((50, 7, 3))


def test_err_zero_for_exact_match(obs):
    e, n = misfit.err(obs, obs)
    assert e == 0.0 and n == 21


def test_err_one_for_zero_prediction(obs):
    assert abs(misfit.err(0 * obs, obs)[0] - 1.0) < 1e-15


def test_err_one_for_doubled_prediction(obs):
    assert abs(misfit.err(2 * obs, obs)[0] - 1.0) < 1e-15


def test_err_scale_invariant(obs):
    U = obs + 0.1 * np.random.default_rng(1).standard_normal(obs.shape)
    assert abs(misfit.err(U, obs)[0] - misfit.err(3.7 * U, 3.7 * obs)[0]) < 1e-14


def test_err_single_pair_value():
    # one receiver, one non-zero component: ERR = ||U - obs|| / ||obs||
    obs = np.zeros((4, 1, 3))
    obs[:, 0, 0] = [3.0, 0.0, 4.0, 0.0]
    U = np.zeros_like(obs)
    U[:, 0, 0] = [0.0, 0.0, 4.0, 0.0]
    e, n = misfit.err(U, obs)
    assert n == 1 and abs(e - 3.0 / 5.0) < 1e-15


def test_err_mean_over_pairs():
    obs = np.ones((10, 2, 3))
    U = obs.copy()
    U[:, 1, 2] = 0.0   # one pair fully wrong -> 1/6
    e, n = misfit.err(U, obs)
    assert n == 6 and abs(e - 1 / 6) < 1e-15
