"""Pins of the SMC-IRMH oracle (independent Metropolis-Hastings inner kernel,
Sec. 2 (ii), App. A) against closed forms, an independent linear-algebra route
and exact evidences."""

import math

import numpy as np
import pytest

import exact
from oracle import irmh, rng
from oracle.action import action


def free_precision(L, m2, beta):
    """I + beta K with K the quadratic form of the free action (lambda = 0),
    S = 1/2 phi^T K phi, K = sum_mu (2 I - T_mu - T_mu^T) + m2 I, built from
    the periodic shift matrices T_mu of the lattice (not from the action code)."""
    d = L * L
    idx = np.arange(d).reshape(L, L)
    K = m2 * np.eye(d)
    for axis in (0, 1):
        T = np.zeros((d, d))
        T[idx.ravel(), np.roll(idx, -1, axis=axis).ravel()] = 1.0   # (T phi)_x = phi_{x+mu}
        K += 2.0 * np.eye(d) - T - T.T
    return np.eye(d) + beta * K


def test_free_precision_matches_action():
    L, m2 = 3, 0.7
    K = free_precision(L, m2, 1.0) - np.eye(L * L)
    phi = np.random.default_rng(0).standard_normal((5, L * L))
    assert np.allclose(0.5 * np.einsum("ni,ij,nj->n", phi, K, phi), action(phi, L, m2, 0.0),
                       rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("L,beta", [(2, 0.3), (3, 0.6), (4, 1.0)])
def test_exact_proposal_always_accepts(L, beta):
    """Proposal = the tempered target itself (free theory): the Hastings ratio
    cancels the target ratio, log alpha = 0 for every pair of fields."""
    m2 = 0.7
    sigma = np.linalg.inv(free_precision(L, m2, beta))
    chol = np.linalg.cholesky(sigma)
    mu = np.zeros(L * L)
    phi = np.random.default_rng(1).standard_normal((64, L * L)) * 1.7 + 0.2
    r = irmh.whitened_sq(phi, mu, chol)
    prop, zz = irmh.propose(mu, chol, 3, 0, 2, 5, np.arange(64))
    la = irmh.log_alpha(phi, prop, r, zz, beta, L, m2, 0.0)
    assert np.max(np.abs(la)) < 1e-10
    # and the step accepts every proposal
    S = action(phi, L, m2, 0.0)
    _, _, r2, acc = irmh.irmh_step(phi, S, r, mu, chol, beta, L, m2, 0.0, 3, 0, 2, 5)
    assert acc.all()
    assert np.allclose(r2, zz)


def test_whitened_residual_is_mahalanobis():
    d = 7
    g = np.random.default_rng(2)
    a = g.standard_normal((d, d))
    sigma = a @ a.T + 0.5 * np.eye(d)
    chol = np.linalg.cholesky(sigma)
    mu = g.standard_normal(d)
    phi = g.standard_normal((11, d))
    x = phi - mu
    maha = np.einsum("ni,ij,nj->n", x, np.linalg.inv(sigma), x)
    assert np.allclose(irmh.whitened_sq(phi, mu, chol), maha, rtol=1e-12)


def test_proposal_moments():
    """phi' = mu + L z has mean mu and covariance L L^T."""
    d = 3
    chol = np.array([[1.0, 0, 0], [0.5, 0.8, 0], [-0.3, 0.2, 0.6]])
    mu = np.array([0.3, -1.0, 2.0])
    n = 40000
    prop, zz = irmh.propose(mu, chol, 7, 1, 1, 0, np.arange(n))
    assert np.allclose(prop.mean(axis=0), mu, atol=5 * 1.1 / math.sqrt(n))
    assert np.allclose(np.cov(prop.T), chol @ chol.T, atol=0.03)
    z = rng.normals(7, 1, 1, 0, rng.PROPOSE, np.arange(n), d)
    assert np.allclose(zz, np.sum(z * z, axis=1))


def test_misfit_proposal_keeps_the_target():
    """Exact samples of a Gaussian target stay distributed as the target under
    an independence sampler with a shifted, widened proposal (detailed balance
    needs the q ratio with the right sign; without it the cloud drifts toward
    the proposal)."""
    L, m2, beta = 2, 0.5, 1.0
    d = L * L
    sigma = np.linalg.inv(free_precision(L, m2, beta))
    ct = np.linalg.cholesky(sigma)
    n = 20000
    phi = np.random.default_rng(3).standard_normal((n, d)) @ ct.T
    mu = np.full(d, 0.6)
    chol = 1.6 * ct
    S = action(phi, L, m2, 0.0)
    r = irmh.whitened_sq(phi, mu, chol)
    for s in range(12):
        phi, S, r, acc = irmh.irmh_step(phi, S, r, mu, chol, beta, L, m2, 0.0, 11, 0, 1, s)
    sd = np.sqrt(np.diag(sigma))
    assert np.all(np.abs(phi.mean(axis=0)) < 5 * sd / math.sqrt(n) * 2.0)
    assert np.allclose(np.var(phi, axis=0), np.diag(sigma), rtol=0.05)
    assert 0.2 < acc.mean() < 0.9


def _replicas(fn, seeds):
    out = [fn(s) for s in seeds]
    z = np.array([o["logz"] for o in out])
    return out, z.mean(), z.std(ddof=1) / math.sqrt(len(z))


def test_smc_irmh_free_2x2():
    _, m, se = _replicas(lambda s: irmh.smc_run(2, 1.0, 0.0, 1024, 0.5, 10, seed=s), range(8))
    assert abs(m - exact.free_logz(2, 1.0)) < 3 * se + 0.01


def test_smc_irmh_free_4x4():
    _, m, se = _replicas(lambda s: irmh.smc_run(4, 1.0, 0.0, 1024, 0.5, 10, seed=s), range(6))
    assert abs(m - exact.free_logz(4, 1.0)) < 3 * se + 0.02


def test_smc_irmh_interacting_2x2_quadrature():
    _, m, se = _replicas(lambda s: irmh.smc_run(2, -4.0, 8.0, 1024, 0.5, 10, seed=s), range(8))
    assert abs(m - exact.logz_2x2(-4.0, 8.0)) < 3 * se + 0.01
