"""Pins of the oracle's covariance estimate and jittered Cholesky factor."""

import numpy as np
import pytest

import synth
from oracle import smc


def test_covariance_matches_numpy_cov():
    phi = synth.fields(3, 500, 4).astype(np.float64) * 2 + 1
    np.testing.assert_allclose(smc.covariance(phi), np.cov(phi, rowvar=False), rtol=1e-12, atol=1e-14)


def test_covariance_needs_two():
    with pytest.raises(ValueError):
        smc.covariance(np.ones((1, 4)))


@pytest.mark.parametrize("d", [1, 4, 16, 64])
def test_factor_reconstructs(d):
    A = synth.spd_matrix(d, d, cond=1e4)
    Lf, tau = smc.cholesky_jitter(A)
    assert np.allclose(Lf, np.tril(Lf)) and np.all(np.diag(Lf) > 0)
    assert tau == pytest.approx(1e-10 * np.trace(A) / d)
    err = np.linalg.norm(Lf @ Lf.T - (A + tau * np.eye(d)))
    assert err <= 1e-12 * np.linalg.norm(A)


def test_rank_deficient_gets_jitter_escalation():
    x = synth.fields(5, 3, 2).astype(np.float64)     # 3 particles, d = 4: rank 2
    A = smc.covariance(x)
    Lf, tau = smc.cholesky_jitter(A)
    assert tau >= 1e-10 * np.trace(A) / 4
    assert np.linalg.norm(Lf @ Lf.T - A) <= 1e-6 * np.linalg.norm(A) + 10 * tau


def test_indefinite_raises():
    A = np.diag([1.0, -1.0, 1.0])
    with pytest.raises(smc.CholeskyError):
        smc.cholesky_jitter(A)
