"""Pins of the SMC-HMC oracle (Hamiltonian Monte Carlo inner kernel,
Sec. 2 (iii), App. A): the action gradient against finite differences and
closed forms, the leapfrog integrator's reversibility and order, stationarity
of an exact Gaussian target, and the full sampler against exact evidences."""

import math

import numpy as np
import pytest

import exact
from oracle import hmc
from oracle.action import action
from test_oracle_irmh import free_precision


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_gradient_matches_central_differences(L):
    g = np.random.default_rng(L)
    phi = g.standard_normal((3, L * L)) * 0.8
    m2, lam = -1.3, 0.7
    grad = hmc.grad_action(phi, L, m2, lam)
    h = 1e-5
    fd = np.empty_like(phi)
    for x in range(L * L):
        e = np.zeros(L * L)
        e[x] = h
        fd[:, x] = (action(phi + e, L, m2, lam) - action(phi - e, L, m2, lam)) / (2 * h)
    assert np.allclose(grad, fd, rtol=1e-7, atol=1e-7)


def test_gradient_of_constant_field():
    """Constant field c: the kinetic part vanishes, dS/dphi = m^2 c + 4 lambda c^3."""
    L, m2, lam, c = 4, -2.0, 0.5, 1.3
    grad = hmc.grad_action(np.full((1, L * L), c), L, m2, lam)
    assert np.allclose(grad, m2 * c + 4 * lam * c ** 3, rtol=1e-14)


def test_gradient_is_free_precision_times_field():
    """lambda = 0: grad (U0 + beta S) = (I + beta K) phi."""
    L, m2, beta = 3, 0.4, 0.7
    phi = np.random.default_rng(9).standard_normal((4, L * L))
    A = free_precision(L, m2, beta)
    assert np.allclose(hmc.grad_potential(phi, beta, L, m2, 0.0), phi @ A.T, rtol=1e-13)


def test_leapfrog_is_reversible():
    L, m2, lam, beta = 3, -1.0, 2.0, 0.8
    g = np.random.default_rng(4)
    phi = g.standard_normal((5, L * L))
    v = 0.5 + g.random(L * L)
    p = g.standard_normal((5, L * L)) / np.sqrt(v)
    phi1, p1 = hmc.leapfrog(phi, p, v, 0.05, 20, beta, L, m2, lam)
    phi2, p2 = hmc.leapfrog(phi1, -p1, v, 0.05, 20, beta, L, m2, lam)
    assert np.allclose(phi2, phi, atol=1e-11)
    assert np.allclose(-p2, p, atol=1e-11)


def test_leapfrog_energy_error_is_second_order():
    """Fixed trajectory length: halving eps cuts |dH| by about 4."""
    L, m2, lam, beta = 3, -1.0, 1.0, 1.0
    g = np.random.default_rng(5)
    phi = g.standard_normal((64, L * L)) * 0.7
    v = np.full(L * L, 0.3)
    p = g.standard_normal((64, L * L)) / np.sqrt(v)
    errs = []
    for eps, n in [(0.04, 10), (0.02, 20), (0.01, 40)]:
        phi1, p1 = hmc.leapfrog(phi, p, v, eps, n, beta, L, m2, lam)
        errs.append(np.mean(np.abs(hmc.hamiltonian_change(phi, p, phi1, p1, v, beta, L, m2,
                                                          lam))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


def test_hmc_keeps_an_exact_gaussian_target():
    """Exact samples of the free-theory target at beta stay so distributed
    under HMC with a mass that does not match the target."""
    L, m2, beta = 2, 0.5, 1.0
    d = L * L
    sigma = np.linalg.inv(free_precision(L, m2, beta))
    n = 20000
    phi = np.random.default_rng(6).standard_normal((n, d)) @ np.linalg.cholesky(sigma).T
    S = action(phi, L, m2, 0.0)
    v = np.full(d, 0.7)
    for s in range(6):
        phi, S, acc = hmc.hmc_step(phi, S, v, 0.5, 7, beta, L, m2, 0.0, 13, 0, 1, s)
    sd = np.sqrt(np.diag(sigma))
    assert np.all(np.abs(phi.mean(axis=0)) < 5 * sd / math.sqrt(n) * 2.0)
    assert np.allclose(np.var(phi, axis=0), np.diag(sigma), rtol=0.05)
    assert 0.5 < acc.mean() < 1.0


def test_leapfrog_conserves_energy_at_small_steps():
    """With the potential's own gradient the energy error of a 20-step
    trajectory at a small step is small (a wrong gradient term or mass scale
    breaks this at once)."""
    L, m2, lam, beta = 3, -1.0, 2.0, 1.0
    g = np.random.default_rng(8)
    phi = g.standard_normal((256, L * L)) * 0.5
    v = np.full(L * L, 0.2)
    p = g.standard_normal((256, L * L)) / np.sqrt(v)
    phi1, p1 = hmc.leapfrog(phi, p, v, 0.05, 20, beta, L, m2, lam)
    dH = hmc.hamiltonian_change(phi, p, phi1, p1, v, beta, L, m2, lam)
    assert np.median(np.abs(dH)) < 0.05


def _replicas(fn, seeds):
    out = [fn(s) for s in seeds]
    z = np.array([o["logz"] for o in out])
    return out, z.mean(), z.std(ddof=1) / math.sqrt(len(z))


def test_smc_hmc_free_2x2():
    _, m, se = _replicas(lambda s: hmc.smc_run(2, 1.0, 0.0, 1024, 0.5, 3, seed=s), range(8))
    assert abs(m - exact.free_logz(2, 1.0)) < 3 * se + 0.01


def test_smc_hmc_free_4x4():
    _, m, se = _replicas(lambda s: hmc.smc_run(4, 1.0, 0.0, 1024, 0.5, 3, seed=s), range(6))
    assert abs(m - exact.free_logz(4, 1.0)) < 3 * se + 0.02


def test_smc_hmc_interacting_2x2_quadrature():
    _, m, se = _replicas(lambda s: hmc.smc_run(2, -4.0, 8.0, 1024, 0.5, 3, seed=s), range(8))
    assert abs(m - exact.logz_2x2(-4.0, 8.0)) < 3 * se + 0.01


def test_smc_hmc_adapts_step_size():
    r = hmc.smc_run(4, -4.0, 8.0, 256, 0.5, 3, seed=0)
    accs = [lv["acc"] for lv in r["levels"]]
    assert all(0.0 <= a <= 1.0 for a in accs)
    assert abs(np.mean(accs[len(accs) // 2:]) - 0.65) < 0.25
