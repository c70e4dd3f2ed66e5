"""Pins of the oracle's random-walk Metropolis step (App. A)."""

import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import action as act
from oracle import rng, smc


def _kinetic_matrix(L):
    d = L * L
    K = np.zeros((d, d))
    for dx0, dx1 in ((1, 0), (0, 1)):
        T = np.zeros((d, d))
        for a in range(L):
            for b in range(L):
                T[a * L + b, ((a + dx0) % L) * L + (b + dx1) % L] = 1.0
        K += (np.eye(d) - T).T @ (np.eye(d) - T)
    return K


def test_gaussian_target_stays_stationary():
    """lambda = 0: p_beta is N(0, C), C = (I + beta (m^2 I + K))^-1; exact draws
    must keep their covariance under the kernel."""
    L, m2, beta, n = 4, 1.0, 0.6, 20000
    d = L * L
    C = np.linalg.inv(np.eye(d) + beta * (m2 * np.eye(d) + _kinetic_matrix(L)))
    cf = np.linalg.cholesky(C)
    phi = synth.rng(11).standard_normal((n, d)) @ cf.T
    S = act.action(phi, L, m2, 0.0)
    B = (2.38 / math.sqrt(d)) * cf
    n_acc = 0
    for s in range(30):
        phi, S, acc = smc.rwmh_step(phi, S, B, beta, L, m2, 0.0, 9, 0, 1, s)
        n_acc += acc.sum()
    assert 0.15 < n_acc / (30 * n) < 0.6
    emp = np.cov(phi, rowvar=False)
    se = np.sqrt((C ** 2 + np.outer(np.diag(C), np.diag(C))) / n)
    assert np.max(np.abs(emp - C) / se) < 5.0
    assert np.all(np.abs(phi.mean(axis=0)) < 5 * np.sqrt(np.diag(C) / n))
    np.testing.assert_allclose(S, act.action(phi, L, m2, 0.0), rtol=1e-12)


def test_one_site_acceptance_probability():
    """d = 1: acceptance from a fixed point equals E_z[min(1, p(x + eps z) / p(x))]."""
    m2, lam, beta, x0, eps, n = -4.0, 8.0, 0.7, 0.4, 0.5, 200000

    def logp(x):
        return -0.5 * x * x - beta * (0.5 * m2 * x * x + lam * x ** 4)

    expect, _ = quad(lambda z: min(1.0, math.exp(logp(x0 + eps * z) - logp(x0)))
                     * math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi), -12, 12)
    phi = np.full((n, 1), x0)
    S = act.action(phi, 1, m2, lam)
    _, _, acc = smc.rwmh_step(phi, S, np.array([[eps]]), beta, 1, m2, lam, 3, 0, 2, 0)
    sd = math.sqrt(expect * (1 - expect) / n)
    assert abs(acc.mean() - expect) < 5 * sd


def test_accept_rule_strict_and_nan():
    assert not smc.accept(0.0, 0.0)
    assert smc.accept(-1e-300, 0.0)
    assert not smc.accept(-1.0, np.nan)


@pytest.mark.parametrize("precision", ["bf16", "fp16", "fp32"])
def test_reduced_precision_increment_is_odd(precision):
    d = 64
    B = synth.lower_factor(3, d, 0.3)
    zero = np.zeros((16, d))
    up = smc.propose(zero, B, 1, 0, 2, 3, np.arange(16), precision, zsign=1.0)
    dn = smc.propose(zero, B, 1, 0, 2, 3, np.arange(16), precision, zsign=-1.0)
    np.testing.assert_array_equal(dn, -up)


def test_proposal_uses_the_propose_stream():
    d = 16
    B = synth.lower_factor(4, d)
    phi = synth.fields(1, 5, 4).astype(np.float64)
    rows = np.array([3, 0, 7, 2, 9])
    prop = smc.propose(phi, B, 5, 1, 4, 6, rows)
    z = rng.normals(5, 1, 4, 6, rng.PROPOSE, rows, d)
    for i in range(5):                       # per-particle matrix-vector route
        np.testing.assert_allclose(prop[i], phi[i] + B @ z[i], rtol=1e-13, atol=1e-13)


def test_eps_adaptation_rule():
    e0 = 0.3
    assert smc.adapt_eps(e0, 30, 100, e0, 0.3) == pytest.approx(e0)
    assert smc.adapt_eps(e0, 100, 100, e0, 0.3) == pytest.approx(e0 * math.exp(0.7))
    assert smc.adapt_eps(e0 / 99, 0, 100, e0, 0.3) == pytest.approx(e0 / 100)
    assert smc.adapt_eps(9.9 * e0, 100, 100, e0, 0.3) == pytest.approx(10 * e0)
