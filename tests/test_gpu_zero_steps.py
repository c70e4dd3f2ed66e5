"""Degenerate case shared by every inner kernel: with zero Metropolis steps per
level (or per nested-sampling refill) a run is the reweight / resample chain
alone, so the random-walk, independence and HMC kernels of SMC (and the
random-walk and slice refills of NS) must give the same run, and the float64
oracle the same log Z."""
import sys

import numpy as np
import pytest

from oracle import ns as ons
from oracle import smc as osmc

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2511_15196_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (with no mutation the resampled cloud shrinks to fewer distinct rows each
# level; larger lattices need more levels and end with a single distinct row,
# whose zero covariance no jitter relative to its trace can factor: the
# documented PHI4_ECHOL, which float64 reaches on that matrix too)
@pytest.mark.parametrize("L,N", [(2, 256), (4, 256)])
def test_smc_zero_steps_same_run_for_every_kernel(L, N):
    say("smc zero steps L", L, "N", N)
    out = {}
    for k in ("rw", "irmh", "hmc"):
        if k == "irmh" and L * L > P.PHI4_IRMH_MAX_SITES:
            continue
        s = P.SMC(L, N, -1.0, 2.0, ess_frac=0.5, n_steps=0, seed=3, kernel=k)
        rc, lv = s.run()
        assert rc == P.PHI4_DONE
        out[k] = (lv, s.logz(), s.phi.cpu().numpy(), s.S.cpu().numpy())
        s.close()
    o = osmc.smc_run(L, -1.0, 2.0, N, 0.5, 0, seed=3)
    say({k: (v[0], v[1]) for k, v in out.items()}, "oracle", o["n_levels"], o["logz"])
    lv0, z0, phi0, S0 = out["rw"]
    for k, (lv, z, phi, S) in out.items():
        assert lv == lv0 == o["n_levels"]
        assert abs(z - z0) < 1e-6 * abs(z0)
        assert np.array_equal(phi, phi0)          # rows are only moved
        assert np.allclose(S, S0, rtol=2e-6, atol=1e-5)
    assert abs(z0 - o["logz"]) < 1e-4 * abs(o["logz"])


def test_ns_zero_steps_same_state_for_both_refills():
    """Four iterations without refill moves: the two refills leave the same
    live points, actions and log Z, bit for bit.  (Run to termination the
    live set collapses onto one field first, whose zero covariance is the
    documented PHI4_ECHOL.)"""
    say("ns zero steps, 4 iterations")
    res = {}
    for k in ("rw", "slice"):
        run = P.NS(4, 200, 100, 0, -1.0, 2.0, prior_var=1.0, term_frac=1e-2, seed=2, kernel=k)
        for _ in range(4):
            P.ns_step(run.h)
        res[k] = (P.logz(run.h)[0], run.phi.cpu().numpy(), run.S.cpu().numpy())
        run.close()
    say("log Z", res["rw"][0], res["slice"][0])
    assert res["rw"][0] == res["slice"][0]
    assert np.array_equal(res["rw"][1], res["slice"][1])
    assert np.array_equal(res["rw"][2], res["slice"][2])
