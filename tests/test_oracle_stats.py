"""Statistical pins of the full oracle samplers against exact evidences.

Seeds are fixed, so every check is deterministic; the tolerances are the
replica standard errors the checks would need if the seeds were drawn at
random.
"""

import math

import numpy as np
import pytest

import exact
from oracle import ns, smc


def _replicas(fn, seeds):
    out = [fn(s) for s in seeds]
    z = np.array([o["logz"] for o in out])
    return out, z.mean(), z.std(ddof=1) / math.sqrt(len(z))


def test_exact_values_self_consistent():
    # the 2x2 transfer-matrix rule reproduces the free closed form
    assert exact.logz_2x2(1.0, 0.0, h=0.05, xmax=8) == pytest.approx(exact.free_logz(2, 1.0), abs=1e-11)
    assert exact.logz_2x2(1.0, 0.0, s2=4.0, h=0.05, xmax=12) == pytest.approx(
        exact.free_logz(2, 1.0, 4.0), abs=1e-11)
    assert exact.logz_1x1(1.0, 0.0) == pytest.approx(exact.free_logz(1, 1.0), abs=1e-12)
    assert exact.free_logz(8, 1.0) == pytest.approx(-55.2738887751, abs=1e-9)


def test_smc_free_2x2():
    _, m, se = _replicas(lambda s: smc.smc_run(2, 1.0, 0.0, 1024, 0.5, 20, seed=s), range(8))
    assert abs(m - exact.free_logz(2, 1.0)) < 3 * se + 0.01


def test_smc_free_4x4_enough_steps():
    _, m, se = _replicas(lambda s: smc.smc_run(4, 1.0, 0.0, 1024, 0.5, 50, seed=s), range(8))
    assert abs(m - exact.free_logz(4, 1.0)) < 3 * se + 0.02


def test_smc_interacting_2x2_quadrature():
    out, m, se = _replicas(lambda s: smc.smc_run(2, -4.0, 8.0, 1024, 0.5, 20, seed=s), range(8))
    assert abs(m - exact.logz_2x2(-4.0, 8.0)) < 3 * se + 0.01


def test_smc_interacting_1x1_quadrature():
    _, m, se = _replicas(lambda s: smc.smc_run(1, -4.0, 1.0, 2048, 0.5, 10, seed=s), range(8))
    assert abs(m - exact.logz_1x1(-4.0, 1.0)) < 3 * se + 0.005


def test_smc_free_magnetisation():
    out, _, _ = _replicas(lambda s: smc.smc_run(2, 1.0, 0.0, 2048, 0.5, 20, seed=s), range(6))
    ms = np.array([o["mean_abs_m"] for o in out])
    se = ms.std(ddof=1) / math.sqrt(len(ms))
    assert abs(ms.mean() - exact.free_mean_abs_m(2, 1.0)) < 3 * se + 0.005


def test_smc_reaches_beta_one_and_adapts():
    r = smc.smc_run(4, -4.0, 8.0, 256, 0.5, 10, seed=0)
    betas = [lv["beta"] for lv in r["levels"]]
    assert betas[-1] == 1.0 and np.all(np.diff(betas) > 0)
    for lv in r["levels"][:-1]:
        assert lv["ess"] >= 0.5 * 256 * (1 - 1e-9)
    assert 0.15 < np.mean([lv["acc"] for lv in r["levels"]]) < 0.45


def test_ns_shrinkage_sequence():
    xs = ns.shrink_sequence(-1.5, 10, 4)
    expect = -1.5 - np.cumsum([1 / 10, 1 / 9, 1 / 8, 1 / 7])
    np.testing.assert_allclose(xs, expect, rtol=1e-15)


def test_ns_deletion_order_ties_by_index():
    logL = np.array([0.5, -1.0, 0.5, -1.0, 2.0])
    np.testing.assert_array_equal(ns.deletion_order(logL), [1, 3, 0, 2, 4])


def test_ns_free_1x1():
    _, m, se = _replicas(lambda s: ns.ns_run(1, 1.0, 0.0, 200, 100, 10, seed=s), range(8))
    assert abs(m - exact.free_logz(1, 1.0, 4.0)) < 3 * se + 0.01


def test_ns_free_2x2():
    out, m, se = _replicas(lambda s: ns.ns_run(2, 1.0, 0.0, 400, 200, 20, seed=s), range(8))
    assert abs(m - exact.free_logz(2, 1.0, 4.0)) < 3 * se + 0.02
    # the sqrt(H/n) error bar is the right size
    assert 0.3 < out[0]["logz_err"] / (se * math.sqrt(8)) < 3.0


def test_ns_interacting_2x2_quadrature():
    _, m, se = _replicas(lambda s: ns.ns_run(2, -4.0, 8.0, 400, 200, 20, seed=s), range(8))
    assert abs(m - exact.logz_2x2(-4.0, 8.0, s2=4.0, xmax=6.0)) < 3 * se + 0.02
