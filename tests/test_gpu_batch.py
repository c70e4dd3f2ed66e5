"""Batched form: many independent SMC runs of different lattice sizes,
couplings and proposal precisions advanced together through one replayed
hipGraph (Sec. 2 tempered SMC, run independently per replica).

Each run in a batch executes exactly the kernels, in exactly the order, of the
same run driven alone, so the batch must reproduce the stand-alone runs bit for
bit: levels, log Z, final particles and actions.  The stand-alone runs are in
turn tied to the float64 oracle by the sampler parity tests.
"""
import pytest
import torch

import paper_2511_15196_amd as P

pytestmark = pytest.mark.gpu

# (L, N, m2, lambda, precision): fused sweeps (d <= 256) and three-pass sweeps
# (d = 289, 324) side by side, float32 and bfloat16 proposal products
RUNS = [
    (4, 256, -4.0, 8.0, "fp32"),
    (8, 1024, -2.0, 4.0, "bf16"),
    (17, 1024, -1.0, 8.0, "fp32"),
    (8, 512, 1.0, 0.0, "fp32"),
    (18, 768, -4.0, 4.0, "bf16"),
]


def make(i, L, N, m2, lam, prec):
    return P.SMC(L, N, m2, lam, ess_frac=0.5, n_steps=10, seed=100 + i, precision=prec)


def alone():
    out = []
    for i, r in enumerate(RUNS):
        s = make(i, *r)
        rc, lv = s.run()
        assert rc == P.PHI4_DONE
        out.append(dict(levels=lv, logz=s.logz(), phi=s.phi.clone(), S=s.S.clone(),
                        m=s.observables()["mean_abs_m"]))
        s.close()
    return out


def check_same(runs, ref):
    for s, r in zip(runs, ref):
        assert s.observables()["levels"] == r["levels"]
        assert s.logz() == r["logz"]
        assert torch.equal(s.phi, r["phi"])
        assert torch.equal(s.S, r["S"])
        assert s.observables()["mean_abs_m"] == r["m"]


def test_batch_reproduces_standalone_runs():
    print("batch vs stand-alone", RUNS, flush=True)
    ref = alone()
    runs = [make(i, *r) for i, r in enumerate(RUNS)]
    rc, levels = P.smc_batch_run([s.h for s in runs])
    assert rc == P.PHI4_DONE
    assert levels == [r["levels"] for r in ref]
    check_same(runs, ref)
    for s in runs:
        s.close()


def test_batch_stops_at_level_cap_and_runs_continue():
    print("batch level cap then smc_run", flush=True)
    ref = alone()
    runs = [make(i, *r) for i, r in enumerate(RUNS)]
    rc, levels = P.smc_batch_run([s.h for s in runs], max_levels=3)
    assert rc == P.PHI4_OK
    assert all(1 <= lv <= 4 for lv in levels)
    for s in runs:
        rc, _ = s.run()
        assert rc == P.PHI4_DONE
    check_same(runs, ref)
    for s in runs:
        s.close()


def test_batch_rejects_bad_handles():
    s = make(0, *RUNS[0])
    with pytest.raises(P.Phi4Error):
        P.smc_batch_run([s.h, s.h])
    s.close()
