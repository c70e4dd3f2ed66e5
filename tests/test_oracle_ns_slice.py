"""Pins of the slice-sampling refill of the nested-sampling oracle (Sec. 2
(iv), App. A; Neal's stepping-out and shrinkage): invariance of the prior and
of the likelihood-constrained prior under the move, the constraint itself, and
the full sampler against exact evidences."""

import math

import numpy as np
from scipy import stats

import exact
from oracle import ns, rng
from oracle.action import action


def _moves(x, S_star, prior_var, L, m2, lam, n_moves, seed, dirs):
    """n_moves slice moves of every row of x (N, d) along the directions dirs(step)."""
    S = action(x, L, m2, lam)
    for s in range(n_moves):
        U = dirs(s)
        for i in range(x.shape[0]):
            def uniforms(q, i=i, s=s):
                return rng.slice_uniform(seed, 0, 1, s, i, q)
            x[i], S[i] = ns.slice_move(x[i], U[i], S[i], S_star, prior_var, L, m2, lam, uniforms)
    return x, S


def test_slice_move_keeps_the_prior():
    """No constraint (S* = inf): a 1-site Gaussian prior N(0, 4) stays so
    distributed, and moves are not trivial."""
    n, s2 = 4000, 4.0
    x0 = np.random.default_rng(1).standard_normal((n, 1)) * 2.0
    x, _ = _moves(x0.copy(), math.inf, s2, 1, 0.0, 0.0, 3, 5,
                  lambda s: rng.normals(5, 0, 1, s, rng.PROPOSE, np.arange(n), 1) * 1.5)
    assert abs(x.mean()) < 4 * 2.0 / math.sqrt(n)
    assert abs(x.var() / s2 - 1.0) < 0.06
    assert np.mean(np.abs(x - x0) > 1e-12) > 0.99
    assert stats.kstest(x[:, 0] / 2.0, "norm").pvalue > 1e-3


def test_slice_move_keeps_the_constrained_prior():
    """L = 1 (no kinetic term): S = m^2 phi^2 / 2 + lambda phi^4, so S < S* is
    |phi| < a; the constrained prior is N(0, s2) truncated to (-a, a), which
    the move must keep, never leaving the constraint."""
    n, s2, m2, lam = 4000, 4.0, 1.0, 0.5
    a = 1.3
    S_star = 0.5 * m2 * a * a + lam * a ** 4
    tn = stats.truncnorm(-a / 2.0, a / 2.0, scale=2.0)
    x0 = tn.rvs(size=(n, 1), random_state=np.random.default_rng(2))
    x, S = _moves(x0.copy(), S_star, s2, 1, m2, lam, 3, 7,
                  lambda s: rng.normals(7, 0, 1, s, rng.PROPOSE, np.arange(n), 1) * 1.0)
    assert np.all(np.abs(x) < a) and np.all(S < S_star)
    assert np.allclose(S, action(x, 1, m2, lam))
    assert abs(x.var() / tn.var() - 1.0) < 0.06
    assert stats.kstest(x[:, 0], tn.cdf).pvalue > 1e-3


def test_slice_move_on_a_lattice_respects_the_constraint():
    L, m2, lam, s2 = 3, -1.0, 2.0, 4.0
    g = np.random.default_rng(3)
    x = g.standard_normal((200, L * L)) * 0.5
    S = action(x, L, m2, lam)
    S_star = float(np.quantile(S, 0.9))
    keep = S < S_star
    x = x[keep]
    cov = np.cov(x.T)
    chol = np.linalg.cholesky(cov)
    n = x.shape[0]
    x1, S1 = _moves(x.copy(), S_star, s2, L, m2, lam, 2, 9,
                    lambda s: rng.normals(9, 0, 1, s, rng.PROPOSE, np.arange(n), L * L) @ chol.T)
    assert np.all(S1 < S_star)
    assert np.allclose(S1, action(x1, L, m2, lam))
    assert np.mean(np.any(x1 != x, axis=1)) > 0.95


def test_ns_slice_free_2x2():
    out = [ns.ns_run(2, 1.0, 0.0, 200, 100, 10, prior_var=4.0, seed=s, refill="slice")
           for s in range(4)]
    z = np.array([o["logz"] for o in out])
    se = z.std(ddof=1) / math.sqrt(len(z))
    assert abs(z.mean() - exact.free_logz(2, 1.0, 4.0)) < 3 * se + 0.05


def test_ns_slice_interacting_2x2_quadrature():
    out = [ns.ns_run(2, -4.0, 8.0, 200, 100, 10, prior_var=1.0, seed=s, refill="slice")
           for s in range(4)]
    z = np.array([o["logz"] for o in out])
    se = z.std(ddof=1) / math.sqrt(len(z))
    assert abs(z.mean() - exact.logz_2x2(-4.0, 8.0)) < 3 * se + 0.05


def test_shrinkage_with_a_coarse_bracket():
    """Directions ten times the slice width: the first draws of a move mostly
    miss, so the shrinkage does the work (it must keep the current point
    inside the bracket); the constrained prior is still kept and nearly every
    point still moves."""
    n, s2, m2, lam = 3000, 4.0, 1.0, 0.5
    a = 1.3
    S_star = 0.5 * m2 * a * a + lam * a ** 4
    tn = stats.truncnorm(-a / 2.0, a / 2.0, scale=2.0)
    x0 = tn.rvs(size=(n, 1), random_state=np.random.default_rng(4))
    x, S = _moves(x0.copy(), S_star, s2, 1, m2, lam, 2, 11,
                  lambda s: np.sign(rng.normals(11, 0, 1, s, rng.PROPOSE, np.arange(n), 1)) * 12.0)
    assert np.all(np.abs(x) < a)
    assert np.mean(np.abs(x - x0) > 1e-12) > 0.97
    assert abs(x.var() / tn.var() - 1.0) < 0.07
    assert stats.kstest(x[:, 0], tn.cdf).pvalue > 1e-3
