"""SMC with the Hamiltonian Monte Carlo inner kernel (SMC-HMC, Sec. 2 (iii);
App. A) on the GPU, against the float64 oracle (oracle/hmc.py) on the same
Philox streams, and against exact evidences.

The GPU integrates the trajectories in float32, the oracle in float64, so the
end points differ at the 1e-6 level and acceptance decisions differ only at
near-ties; coupled runs agree in their level counts and closely in log Z.
"""
import math
import sys

import numpy as np
import pytest

import exact
from oracle import hmc as ohmc
from threadpoolctl import threadpool_limits

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2511_15196_amd")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_hmc(L, m2, lam, N, ess, steps, seed, **kw):
    with threadpool_limits(limits=1):
        return ohmc.smc_run(L, m2, lam, N, ess, steps, seed=seed, **kw)


def gpu_hmc(L, N, m2, lam, ess, steps, seed, max_levels=100000, keep=False):
    run = P.SMC(L, N, m2, lam, ess_frac=ess, n_steps=steps, seed=seed, kernel="hmc")
    rc, levels = run.run(max_levels)
    obs = run.observables()
    out = dict(logz=run.logz(), levels=levels, mean_abs_m=obs["mean_abs_m"], acc=obs["acc"],
               eps=obs["eps"], rc=rc)
    if keep:
        out["phi"] = run.phi.cpu().numpy().astype(np.float64)
    run.close()
    return out


@pytest.mark.parametrize("L,N,m2,lam,ess,steps,seeds", [
    (4, 256, -1.0, 2.0, 0.5, 3, 8),
    (4, 256, -4.0, 8.0, 0.5, 3, 8),
    (8, 512, -1.0, 2.0, 0.5, 3, 6),
    (4, 512, -4.0, 1.0, 0.9, 5, 6),   # the paper's point (m0^2 = -4, lambda = 1, ESS 0.9)
])
def test_hmc_replicas_match_oracle(L, N, m2, lam, ess, steps, seeds):
    """Whole runs: one flipped near-tie decision changes the next level's
    adapted step slightly, and 20-step trajectories amplify that until the
    float32 and float64 runs of one seed decouple; replica means of log Z and
    <|M|> then agree within their standard errors."""
    say("hmc replicas L", L, "N", N, "m2", m2, "lambda", lam, "ess", ess)
    g = [gpu_hmc(L, N, m2, lam, ess, steps, s) for s in range(seeds)]
    o = [oracle_hmc(L, m2, lam, N, ess, steps, s) for s in range(seeds)]
    for key in ("logz", "mean_abs_m"):
        a = np.array([r[key] for r in g])
        b = np.array([r[key] for r in o])
        se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
        say(key, "gpu", a.mean(), "oracle", b.mean(), "se", se)
        assert abs(a.mean() - b.mean()) < 3 * se + 1e-3
    assert all(r["rc"] == P.PHI4_DONE for r in g)


def test_hmc_strong_coupling_coupled_to_oracle():
    """lambda = 8: the adapted step sits near the leapfrog stability limit of
    the quartic term, where 20-step trajectories amplify the float32 /
    float64 difference and some decisions flip; the runs stay close."""
    say("hmc L=4 N=256 m2=-4 lambda=8")
    g = gpu_hmc(4, 256, -4.0, 8.0, 0.5, 3, 0)
    o = oracle_hmc(4, -4.0, 8.0, 256, 0.5, 3, 0)
    say("gpu", g, "oracle", o["logz"], o["n_levels"], o["mean_abs_m"])
    assert g["rc"] == P.PHI4_DONE
    assert abs(g["levels"] - o["n_levels"]) <= 1
    assert abs(g["logz"] - o["logz"]) < 0.15
    assert abs(g["mean_abs_m"] - o["mean_abs_m"]) < 0.02


@pytest.mark.parametrize("L,N,steps,tol", [(8, 1024, 3, 0.15)])
def test_hmc_full_runs_coupled_to_oracle(L, N, steps, tol):
    say("hmc coupled L", L, "N", N)
    g = gpu_hmc(L, N, -1.0, 2.0, 0.5, steps, 3)
    o = oracle_hmc(L, -1.0, 2.0, N, 0.5, steps, 3)
    say("gpu", g, "oracle", o["logz"], o["n_levels"], o["mean_abs_m"])
    assert g["rc"] == P.PHI4_DONE
    assert abs(g["levels"] - o["n_levels"]) <= 1
    assert abs(g["logz"] - o["logz"]) < tol
    assert abs(g["mean_abs_m"] - o["mean_abs_m"]) < 0.01


@pytest.mark.parametrize("L,N", [(3, 200), (10, 300), (16, 128), (24, 128), (40, 96), (64, 64)])
def test_hmc_first_levels_track_oracle(L, N):
    """Two levels at every workgroup shape of the kernel (64 .. 1024 threads,
    1, 2 and 4 sites per thread; d = 9, 100, 256, 576, 1600, 4096): log Z
    after two levels, the step adapted after the first and the particles
    themselves against the oracle."""
    say("hmc first levels L", L, "N", N)
    g = gpu_hmc(L, N, -1.0, 2.0, 0.5, 2, 7, max_levels=2, keep=True)
    o = oracle_hmc(L, -1.0, 2.0, N, 0.5, 2, 7, stop_after=2, keep_particles=True)
    diff = np.max(np.abs(g["phi"] - o["phi"]), axis=1)
    frac = np.mean(diff < 1e-3)
    say("logz", g["logz"], o["logz"], "levels", g["levels"], o["n_levels"],
        "rows within 1e-3", frac, "max", diff.max())
    assert g["levels"] == o["n_levels"] == 2
    assert abs(g["logz"] - o["logz"]) < 1e-3 * max(1.0, abs(o["logz"]))
    assert g["eps"] == pytest.approx(o["levels"][-1]["eps"], rel=1e-5)
    assert frac >= 0.95


def test_hmc_free_2x2_exact():
    say("hmc free 2x2 replicas")
    z = np.array([gpu_hmc(2, 2048, 1.0, 0.0, 0.5, 3, s)["logz"] for s in range(8)])
    se = z.std(ddof=1) / math.sqrt(len(z))
    say("mean", z.mean(), "se", se, "exact", exact.free_logz(2, 1.0))
    assert abs(z.mean() - exact.free_logz(2, 1.0)) < 3 * se + 0.01


def test_hmc_rejects_bad_configurations():
    with pytest.raises(P.Phi4Error):
        P.SMC(4, 256, -4.0, 8.0, kernel="hmc", precision="bf16")
    with pytest.raises(P.Phi4Error):
        P.SMC(4, 256, -4.0, 8.0, kernel="hmc", n_leapfrog=-1)


def test_hmc_in_a_batch_matches_standalone():
    """HMC runs inside the replayed graph of the batched form reproduce their
    stand-alone runs bit for bit, next to a random-walk and an IRMH run."""
    say("hmc batch vs stand-alone")
    cfgs = [dict(L=8, N=1024, m2=-2.0, lam=4.0, kernel="hmc"),
            dict(L=4, N=256, m2=-4.0, lam=8.0, kernel="rw"),
            dict(L=6, N=512, m2=-1.0, lam=2.0, kernel="irmh"),
            dict(L=20, N=256, m2=-1.0, lam=2.0, kernel="hmc")]

    def make(i, c):
        return P.SMC(c["L"], c["N"], c["m2"], c["lam"], ess_frac=0.5, n_steps=3, seed=60 + i,
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
