"""SMC with the independent Metropolis-Hastings inner kernel (SMC-IRMH,
Sec. 2 (ii); App. A) on the GPU, against the float64 oracle (oracle/irmh.py)
on the same Philox streams, and against exact evidences.

The GPU forms the mean, the explicit inverse factor and the whitened
residuals on its own (float32 products of float64 factors), so acceptance
decisions can differ from the oracle's only where log u and log alpha are
within rounding of each other; the coupled runs then agree in their level
count and closely in log Z and <|M|>.
"""
import math
import sys

import numpy as np
import pytest

import exact
from oracle import irmh as oirmh
from threadpoolctl import threadpool_limits

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2511_15196_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_irmh(L, m2, lam, N, ess, steps, seed):
    # one BLAS thread: the oracle's small products slow down many times over
    # when the library spreads them over every core
    with threadpool_limits(limits=1):
        return oirmh.smc_run(L, m2, lam, N, ess, steps, seed=seed)


def gpu_irmh(L, N, m2, lam, ess, steps, seed):
    run = P.SMC(L, N, m2, lam, ess_frac=ess, n_steps=steps, seed=seed, kernel="irmh")
    rc, levels = run.run()
    obs = run.observables()
    z = run.logz()
    run.close()
    return dict(logz=z, levels=levels, mean_abs_m=obs["mean_abs_m"], acc=obs["acc"], rc=rc)


@pytest.mark.parametrize("seed", [0, 1])
def test_irmh_small_coupled_to_oracle(seed):
    say("irmh L=4 N=256 seed", seed)
    g = gpu_irmh(4, 256, -4.0, 8.0, 0.5, 10, seed)
    o = oracle_irmh(4, -4.0, 8.0, 256, 0.5, 10, seed)
    say("gpu", g, "oracle", o["logz"], o["n_levels"], o["mean_abs_m"])
    assert g["rc"] == P.PHI4_DONE
    assert g["levels"] == o["n_levels"]
    assert abs(g["logz"] - o["logz"]) < 0.05
    assert abs(g["mean_abs_m"] - o["mean_abs_m"]) < 0.01


def test_irmh_paper_settings_coupled_to_oracle():
    """m0^2 = -4, lambda = 1, ESS 0.9, 3V steps per level (App. A), 4 x 4."""
    say("irmh paper settings L=4 N=512")
    g = gpu_irmh(4, 512, -4.0, 1.0, 0.9, 48, 0)
    o = oracle_irmh(4, -4.0, 1.0, 512, 0.9, 48, 0)
    say("gpu", g, "oracle", o["logz"], o["n_levels"], o["mean_abs_m"])
    assert g["rc"] == P.PHI4_DONE
    assert abs(g["levels"] - o["n_levels"]) <= 1
    assert abs(g["logz"] - o["logz"]) < 0.1
    assert abs(g["mean_abs_m"] - o["mean_abs_m"]) < 0.02


@pytest.mark.parametrize("L,N", [(8, 1024), (10, 1024)])
def test_irmh_whitening_sizes_coupled_to_oracle(L, N):
    """d = 64 and 100: several 64-wide tiles of the whitening product and of
    the inverse factor, the second with a ragged tail."""
    say("irmh coupled L", L, "N", N)
    g = gpu_irmh(L, N, -1.0, 2.0, 0.5, 10, 3)
    o = oracle_irmh(L, -1.0, 2.0, N, 0.5, 10, 3)
    say("gpu", g, "oracle", o["logz"], o["n_levels"], o["mean_abs_m"])
    assert g["rc"] == P.PHI4_DONE
    assert abs(g["levels"] - o["n_levels"]) <= 1
    assert abs(g["logz"] - o["logz"]) < 0.15
    assert abs(g["mean_abs_m"] - o["mean_abs_m"]) < 0.01


def test_irmh_free_2x2_exact():
    say("irmh free 2x2 replicas")
    z = np.array([gpu_irmh(2, 2048, 1.0, 0.0, 0.5, 10, s)["logz"] for s in range(8)])
    se = z.std(ddof=1) / math.sqrt(len(z))
    say("mean", z.mean(), "se", se, "exact", exact.free_logz(2, 1.0))
    assert abs(z.mean() - exact.free_logz(2, 1.0)) < 3 * se + 0.01


def test_irmh_d256_coupled_to_oracle():
    """d = 256 with a well-conditioned cloud (N = 16 d).  With a few
    particles per site the resampled cloud is nearly degenerate (covariance
    condition numbers of 1e6 .. 1e10) and the float32 covariance, like the
    paper's, differs from the oracle's float64 one in its smallest
    directions, so coupled runs separate there; the whitening itself is
    pinned exactly by test_whiten_matches_oracle."""
    say("irmh coupled L 16 N 4096 steps 2")
    g = gpu_irmh(16, 4096, -1.0, 2.0, 0.5, 2, 5)
    o = oracle_irmh(16, -1.0, 2.0, 4096, 0.5, 2, 5)
    say("gpu", g, "oracle", o["logz"], o["n_levels"], o["mean_abs_m"])
    assert g["rc"] == P.PHI4_DONE
    assert abs(g["levels"] - o["n_levels"]) <= 1
    # float32 actions flip a few near-tie decisions, and an independence
    # proposal that is taken or not moves a particle far: the tolerance of
    # the random-walk sampler's coupled large-lattice check
    assert abs(g["logz"] - o["logz"]) < 0.5
    assert abs(g["mean_abs_m"] - o["mean_abs_m"]) < 0.01


@pytest.mark.parametrize("d,N,mapped", [(16, 300, True), (100, 300, False), (256, 777, True),
                                        (400, 513, True), (576, 600, False), (1024, 1100, True)])
def test_whiten_matches_oracle(d, N, mapped):
    """Mean, inverse factor and whitened residuals (float64 on both sides)
    at every register layout of the inverse (1 .. 16 entries per lane), with
    ragged particle and column tails, through a resampling-like row map, for
    a covariance with condition number 1e6."""
    say("whiten d", d, "N", N, "mapped", mapped)
    g = np.random.default_rng(d)
    q, _ = np.linalg.qr(g.standard_normal((d, d)))
    sigma = (q * np.logspace(-6, 0, d)) @ q.T
    chol = np.linalg.cholesky(sigma)
    phi = (g.standard_normal((N, d)) * 2.0 + 0.3).astype(np.float32)
    rows = g.integers(0, N, N).astype(np.int32) if mapped else None
    sel = phi[rows] if mapped else phi
    with threadpool_limits(limits=1):
        mu_o = oirmh.particle_mean(sel.astype(np.float64))
        r_o = oirmh.whitened_sq(sel.astype(np.float64), mu_o, chol)
    dev = torch.device("cuda")
    raw, wsp = P._workspace(P.phi4_whiten_workspace_bytes(N, d), dev)
    r = torch.empty(N, dtype=torch.float32, device=dev)
    mu = torch.empty(d, dtype=torch.float32, device=dev)
    P.phi4_whiten(torch.from_numpy(phi).to(dev), N, d, torch.from_numpy(chol).to(dev), r, wsp,
                  rows=torch.from_numpy(rows).to(dev) if mapped else None, mu=mu)
    torch.cuda.synchronize()
    r_g, mu_g = r.cpu().numpy().astype(np.float64), mu.cpu().numpy().astype(np.float64)
    say("max rel err r", np.max(np.abs(r_g - r_o) / r_o), "mu", np.max(np.abs(mu_g - mu_o)))
    assert np.allclose(r_g, r_o, rtol=1e-6, atol=0)
    assert np.allclose(mu_g, mu_o, rtol=1e-6, atol=1e-7)


def test_irmh_largest_lattice_runs():
    """d = 1024, the largest lattice the independence sampler takes: the run
    reaches beta = 1 with a finite log Z and a nondegenerate acceptance."""
    say("irmh L=32 N=4096")
    g = gpu_irmh(32, 4096, 1.0, 0.0, 0.5, 2, 0)
    say("gpu", g)
    assert g["rc"] == P.PHI4_DONE
    assert math.isfinite(g["logz"])
    assert 0.0 < g["acc"] < 1.0


def test_whiten_rejects_bad_shapes():
    assert P.phi4_whiten_workspace_bytes(10, 1025) == 0
    assert P.phi4_whiten_workspace_bytes(0, 16) == 0
    assert P.phi4_whiten_workspace_bytes(10, 16) > 0


def test_irmh_rejects_reduced_precision_and_large_lattices():
    with pytest.raises(P.Phi4Error):
        P.SMC(4, 256, -4.0, 8.0, kernel="irmh", precision="bf16")
    with pytest.raises(P.Phi4Error):
        P.SMC(33, 256, -4.0, 8.0, kernel="irmh")


def test_irmh_in_a_batch_matches_standalone():
    """An independence-sampler run inside the replayed graph of the batched
    form reproduces its stand-alone run bit for bit, next to a random-walk run."""
    say("irmh batch vs stand-alone")
    cfgs = [dict(L=8, N=1024, m2=-2.0, lam=4.0, kernel="irmh"),
            dict(L=4, N=256, m2=-4.0, lam=8.0, kernel="rw"),
            dict(L=18, N=512, m2=-1.0, lam=2.0, kernel="irmh")]

    def make(i, c):
        return P.SMC(c["L"], c["N"], c["m2"], c["lam"], ess_frac=0.5, n_steps=6, seed=40 + i,
                     kernel=c["kernel"])

    ref = []
    for i, c in enumerate(cfgs):
        s = make(i, c)
        rc, lv = s.run()
        assert rc == P.PHI4_DONE
        ref.append((lv, s.logz(), s.phi.clone()))
        s.close()
    runs = [make(i, c) for i, c in enumerate(cfgs)]
    rc, levels = P.smc_batch_run([s.h for s in runs])
    assert rc == P.PHI4_DONE
    for s, (lv, z, phi), got in zip(runs, ref, levels):
        assert got == lv
        assert s.logz() == z
        assert torch.equal(s.phi, phi)
        s.close()
