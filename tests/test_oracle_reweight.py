"""Pins of the oracle's log-sum-exp, ESS and adaptive beta solve."""

import math

import numpy as np
import pytest
from scipy.special import logsumexp

import synth
from oracle import smc


def test_lse_constant_and_library():
    assert smc.lse(np.full(1000, -3.5)) == pytest.approx(-3.5 + math.log(1000), rel=1e-15)
    a = synth.log_weights(1, 5000, spread=50.0)
    assert smc.lse(a) == pytest.approx(float(logsumexp(a)), rel=1e-14)


def test_ess_limits():
    assert smc.ess(np.zeros(777)) == pytest.approx(777, rel=1e-13)
    one_hot = np.full(10, -np.inf)
    one_hot[3] = 0.0
    assert smc.ess(one_hot) == pytest.approx(1.0)
    w = np.exp(synth.log_weights(2, 100))
    assert smc.ess(np.log(w)) == pytest.approx(w.sum() ** 2 / (w * w).sum(), rel=1e-12)


def _grid_dbeta(S, beta, target, n_grid=20001):
    grid = np.linspace(0.0, 1.0 - beta, n_grid)
    ok = [g for g in grid if smc.ess(-g * S) >= target]
    return max(ok), grid[1] - grid[0]


@pytest.mark.parametrize("beta", [0.0, 0.3, 0.9])
def test_bisection_vs_grid(beta):
    S = 40.0 + 15.0 * np.random.default_rng(7).standard_normal(512)
    target = 0.5 * 512
    db = smc.solve_dbeta(S, beta, target)
    g, h = _grid_dbeta(S, beta, target)
    if db < 1 - beta:
        assert abs(db - g) <= h
        assert smc.ess(-db * S) >= target
        assert smc.ess(-(db * (1 + 1e-9)) * S) < target * (1 + 1e-6)


def test_full_step_when_room_suffices():
    S = np.full(100, 3.0) + 1e-3 * np.arange(100)
    db, nb, dlogz, w = smc.reweight(S, 0.25, 0.5)
    assert db == 0.75 and nb == 1.0
    assert dlogz == pytest.approx(smc.lse(-0.75 * S) - math.log(100))


def test_constant_action_increment():
    S = np.full(64, 2.5)
    db, nb, dlogz, w = smc.reweight(S, 0.0, 0.5)
    assert nb == 1.0 and dlogz == pytest.approx(-2.5, rel=1e-14)
    assert np.all(w == 1.0)


def test_weights_normalised_to_max_one():
    S = 100.0 * np.random.default_rng(1).standard_normal(300)
    db, nb, dlogz, w = smc.reweight(S, 0.0, 0.5)
    assert w.max() == 1.0 and nb < 1.0
    assert smc.ess(np.log(w)) >= 150 * (1 - 1e-9)
