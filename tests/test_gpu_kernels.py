"""GPU parity of the step-level kernels against the FP64 oracle.

Every case runs the HIP kernels through the C ABI (paper_2511_15196_amd) on
seeded inputs from tests/synth.py and compares element by element with the
oracle on the same inputs.
"""

import math
import sys

import numpy as np
import pytest

import synth
from oracle import action as oact
from oracle import precision as oprec
from oracle import rng as orng
from oracle import smc as osmc

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2511_15196_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def ws(nbytes):
    return P._workspace(nbytes, DEV)


# ------------------------------------------------------------------ normals

@pytest.mark.parametrize("purpose,level,step", [(orng.PROPOSE, 3, 7), (orng.INIT, 0, 0)])
def test_normals_match_oracle(purpose, level, step):
    n, d = 777, 64
    say("normals", purpose, level, step)
    out = torch.empty((n, d), dtype=torch.float32, device=DEV)
    P.phi4_normals(11, 2, level, step, purpose, n, d, out)
    got = host(out).astype(np.float64)
    want = orng.normals(11, 2, level, step, purpose, np.arange(n), d)
    err = np.abs(got - want)
    say("max abs err", err.max(), "max rel", (err / (np.abs(want) + 1e-3)).max())
    assert np.all(err <= 2e-6 * (1.0 + np.abs(want)))


def test_normals_rows_and_ragged_d():
    rows = np.array([5, 0, 123456, 7], dtype=np.int32)
    d = 10
    out = torch.empty((4, d), dtype=torch.float32, device=DEV)
    P.phi4_normals(3, 0, 9, 1, orng.PROPOSE, 4, d, out, rows=dev(rows))
    want = orng.normals(3, 0, 9, 1, orng.PROPOSE, rows, d)
    assert np.allclose(host(out), want, atol=2e-6 * 6, rtol=0)


# ------------------------------------------------------------------- action

@pytest.mark.parametrize("L", [1, 2, 3, 4, 8, 10, 16])
def test_action_matches_oracle(L):
    m2, lam = -4.0, 8.0
    phi = synth.broken_phase_fields(L, 301, L)
    say("action L", L)
    S = torch.empty(301, dtype=torch.float32, device=DEV)
    M = torch.empty(301, dtype=torch.float32, device=DEV)
    P.phi4_action(dev(phi), 301, L, m2, lam, S, M)
    p64 = phi.astype(np.float64)
    want = oact.action(p64, L, m2, lam)
    scale = oact.abs_site_sum(p64, L, m2, lam)
    got = host(S).astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-5 * scale)
    np.testing.assert_allclose(host(M), np.abs(oact.magnetisation(p64)), rtol=1e-5, atol=1e-7)


def test_action_z2_bitwise_and_empty():
    L = 16
    phi = synth.fields(5, 64, L)
    S1 = torch.empty(64, dtype=torch.float32, device=DEV)
    S2 = torch.empty(64, dtype=torch.float32, device=DEV)
    P.phi4_action(dev(phi), 64, L, -4.0, 5.0, S1)
    P.phi4_action(dev(-phi), 64, L, -4.0, 5.0, S2)
    assert np.array_equal(host(S1), host(S2))
    P.phi4_action(dev(phi), 0, L, -4.0, 5.0, S1)      # empty launch is a no-op


# -------------------------------------------------------------- resampling

@pytest.mark.parametrize("n", [1, 2, 7, 1000, 4096, 16384])
def test_resample_bit_exact(n):
    say("resample", n)
    w = np.exp(synth.log_weights(n + 1, n, spread=2.5))
    raw, wsp = ws(P.phi4_step_workspace_bytes(n, 0))
    anc = torch.empty(n, dtype=torch.int32, device=DEV)
    for U in (0, 0x9E3779B9, 0xFFFFFFFF):
        P.phi4_resample_systematic(dev(w), n, U, anc, wsp)
        np.testing.assert_array_equal(host(anc), osmc.systematic_resample(w, U))


def test_resample_special_weights():
    n = 513
    raw, wsp = ws(P.phi4_step_workspace_bytes(n, 0))
    anc = torch.empty(n, dtype=torch.int32, device=DEV)
    P.phi4_resample_systematic(dev(np.ones(n)), n, 12345, anc, wsp)
    np.testing.assert_array_equal(host(anc), np.arange(n))
    w = np.zeros(n)
    w[300] = 1e-300
    P.phi4_resample_systematic(dev(w), n, 777, anc, wsp)
    assert np.all(host(anc) == 300)
    with pytest.raises(P.Phi4Error):
        P.phi4_resample_systematic(dev(np.zeros(n)), n, 1, anc, wsp)
    w[5] = np.nan
    with pytest.raises(P.Phi4Error):
        P.phi4_resample_systematic(dev(w), n, 1, anc, wsp)


# ------------------------------------------------------------- reweighting

@pytest.mark.parametrize("n,beta,frac", [(256, 0.0, 0.5), (4096, 0.0, 0.5), (4096, 0.37, 0.9),
                                         (16384, 0.8, 0.5), (1000, 0.999, 0.5)])
def test_reweight_matches_oracle(n, beta, frac):
    say("reweight", n, beta, frac)
    S = (200.0 + 40.0 * synth.rng(n).standard_normal(n)).astype(np.float32)
    raw, wsp = ws(P.phi4_step_workspace_bytes(n, 0))
    w = torch.empty(n, dtype=torch.float64, device=DEV)
    out = P.phi4_reweight(dev(S), n, beta, frac, wsp, w=w)
    db, nb, dlogz, wo = osmc.reweight(S.astype(np.float64), beta, frac)
    say(out, db, nb, dlogz)
    assert out["dbeta"] == pytest.approx(db, rel=1e-12, abs=1e-300)
    assert out["dbeta"] <= 1.0 - beta
    assert out["beta"] == pytest.approx(nb, rel=1e-13)
    assert out["dlogz"] == pytest.approx(dlogz, rel=1e-11, abs=1e-11)
    assert out["ess"] >= frac * n * (1 - 1e-12)
    np.testing.assert_allclose(host(w), wo, rtol=1e-10, atol=1e-300)


def test_reweight_full_step_and_constant():
    n = 64
    raw, wsp = ws(P.phi4_step_workspace_bytes(n, 0))
    out = P.phi4_reweight(dev(np.full(n, 3.5, dtype=np.float32)), n, 0.25, 0.5, wsp)
    assert out["dbeta"] == 0.75 and out["beta"] == 1.0
    assert out["dlogz"] == pytest.approx(-0.75 * 3.5, rel=1e-14)
    with pytest.raises(P.Phi4Error):
        bad = np.full(n, 1.0, dtype=np.float32)
        bad[3] = np.inf
        P.phi4_reweight(dev(bad), n, 0.0, 0.5, wsp)


# ------------------------------------------------- covariance and Cholesky

@pytest.mark.parametrize("n,L", [(2, 2), (100, 4), (4096, 8), (3000, 10), (16384, 16)])
def test_covariance_matches_oracle(n, L):
    d = L * L
    say("cov", n, d)
    phi = (1.5 + synth.fields(n + d, n, L, scale=0.7)).astype(np.float32)
    raw, wsp = ws(P.phi4_step_workspace_bytes(n, d))
    sig = torch.empty((d, d), dtype=torch.float64, device=DEV)
    P.phi4_covariance(dev(phi), n, d, sig, wsp)
    want = osmc.covariance(phi.astype(np.float64))
    got = host(sig)
    assert np.allclose(got, got.T)
    assert np.max(np.abs(got - want)) <= 2e-5 * np.max(np.abs(np.diag(want)))


def test_covariance_row_subset():
    n, L = 500, 4
    d = L * L
    phi = synth.fields(9, n, L)
    rows = np.sort(synth.rng(10).choice(n, 300, replace=False)).astype(np.int32)[::-1].copy()
    raw, wsp = ws(P.phi4_step_workspace_bytes(n, d))
    sig = torch.empty((d, d), dtype=torch.float64, device=DEV)
    P.phi4_covariance(dev(phi), 300, d, sig, wsp, rows=dev(rows))
    want = osmc.covariance(phi[rows].astype(np.float64))
    assert np.max(np.abs(host(sig) - want)) <= 2e-5 * np.max(np.diag(want))


@pytest.mark.parametrize("d,cond", [(1, 1.0), (16, 1e3), (64, 1e4), (100, 1e2), (256, 1e3),
                                    (300, 1e3), (1024, 1e2), (2100, 1e2), (4096, 1e2)])
def test_cholesky_matches_oracle(d, cond):
    say("chol", d)
    A = synth.spd_matrix(d + 1, d, cond=cond)
    raw, wsp = ws(P.phi4_step_workspace_bytes(2, d))
    Lt = torch.empty((d, d), dtype=torch.float64, device=DEV)
    tau = P.phi4_cholesky(dev(A), d, Lt, wsp)
    want, tau0 = osmc.cholesky_jitter(A)
    assert tau == pytest.approx(tau0, rel=1e-14)
    got = host(Lt)
    assert np.allclose(np.triu(got, 1), 0.0)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.sqrt(np.max(np.diag(A))) * d


def test_cholesky_jitter_and_failure():
    d = 16
    x = synth.fields(4, 5, 4).astype(np.float64)       # rank 4 < 16
    A = osmc.covariance(x)
    raw, wsp = ws(P.phi4_step_workspace_bytes(2, d))
    Lt = torch.empty((d, d), dtype=torch.float64, device=DEV)
    tau = P.phi4_cholesky(dev(A), d, Lt, wsp)
    want, tau0 = osmc.cholesky_jitter(A)
    assert tau == pytest.approx(tau0, rel=1e-12)
    with pytest.raises(P.Phi4Error) as e:
        P.phi4_cholesky(dev(np.diag([1.0, -1.0, 2.0])), 3, Lt, wsp)
    assert e.value.code == P.PHI4_ECHOL


@pytest.mark.parametrize("d", [100, 324, 1156])
def test_blocked_cholesky_jitter_escalation(d):
    """Rank-deficient covariance (d > 64): the blocked first attempt fails and
    the escalation reaches the oracle's tau and factor."""
    L = int(round(d ** 0.5))
    x = synth.fields(5, d // 2, L).astype(np.float64)    # rank d/2 - 1 < d
    A = osmc.covariance(x)
    raw, wsp = ws(P.phi4_step_workspace_bytes(2, d))
    Lt = torch.empty((d, d), dtype=torch.float64, device=DEV)
    tau = P.phi4_cholesky(dev(A), d, Lt, wsp)
    want, tau0 = osmc.cholesky_jitter(A)
    say("tau", tau, tau0)
    assert tau == pytest.approx(tau0, rel=1e-12)
    got = host(Lt)
    assert np.allclose(np.triu(got, 1), 0.0)
    assert np.max(np.abs(got - want)) <= 1e-8 * np.sqrt(np.max(np.diag(A))) * d
