"""GPU parity of the random-walk Metropolis sweep against the oracle.

Lattices up to d = 256 run the fused register-resident sweep; larger ones
(d = 324, 576, 1024 here, with ragged 64 x 64 tiles) run the three-pass
form (normals, proposal product, accept); both are held to the same bars.

The proposal product is checked against the oracle's float64 product of the
same (rounded) operands, the Metropolis decisions against the oracle's
float64 decisions on identical phi, phi' and u, and multi-step sweeps
against the oracle stepping the same Philox streams.
"""

import math
import sys

import numpy as np
import pytest

import synth
from oracle import action as oact
from oracle import ns as ons
from oracle import precision as oprec
from oracle import rng as orng
from oracle import smc as osmc

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2511_15196_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda"
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def factor(L, seed, scale=0.6):
    d = L * L
    Lc = synth.lower_factor(seed, d, scale=scale)
    eps = 2.38 / math.sqrt(d)
    Bt32 = np.ascontiguousarray((eps * Lc).T).astype(np.float32)   # Bt[k][c] = eps L[c][k]
    return Bt32, Bt32.T.astype(np.float64)                          # (kernel input, B = eps L)


def run_kernel(phi, L, Bt32, kind=0, beta=0.6, s_star=0.0, prior_var=4.0, seed=5, run=1,
               level=3, step0=2, n_steps=1, zsign=1.0, precision="fp32", rows=None,
               inplace=False, m2=-4.0, lam=8.0):
    n = phi.shape[0] if rows is None else len(rows)
    d = L * L
    src = dev(phi)
    dst = src if inplace else torch.zeros_like(src)
    S = torch.zeros(phi.shape[0], dtype=torch.float32, device=DEV)
    absM = torch.zeros(phi.shape[0], dtype=torch.float32, device=DEV)
    acc = torch.zeros(1, dtype=torch.int64, device=DEV)
    flags = torch.zeros(max(n, 1), dtype=torch.uint8, device=DEV)
    prop = torch.zeros((max(n, 1), d), dtype=torch.float32, device=DEV)
    P.phi4_mutate(src, dst, n, L, m2, lam, dev(Bt32), kind, beta, s_star, prior_var, seed, run,
                  level, step0, n_steps, zsign, PREC[precision], S, absM=absM, acc_count=acc,
                  acc_flags=flags, prop=prop, rows=None if rows is None else dev(rows))
    return dict(dst=host(dst), S=host(S), absM=host(absM), acc=int(host(acc)[0]),
                flags=host(flags)[:n].astype(bool), prop=host(prop)[:n])


def gpu_normals(seed, run, level, step, n, d, rows=None):
    out = torch.empty((max(n, 1), d), dtype=torch.float32, device=DEV)
    P.phi4_normals(seed, run, level, step, orng.PROPOSE, n, d, out,
                   rows=None if rows is None else dev(np.asarray(rows, dtype=np.int32)))
    return host(out)[:n].astype(np.float64)


def product_tolerance(z, B, prop):
    d = B.shape[0]
    mag = np.abs(z) @ np.abs(B).T
    return 4 * d * 2.0 ** -24 * mag + 2.0 ** -23 * np.abs(prop) + 1e-30


@pytest.mark.parametrize("L,n", [(1, 33), (2, 50), (4, 256), (8, 1000), (10, 300), (16, 517),
                                 (17, 90), (18, 70), (32, 130)])
@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_proposal_product(L, n, precision):
    """phi' - phi = B z on MFMA vs the float64 product of the same rounded operands."""
    d = L * L
    say("proposal", L, n, precision)
    phi = synth.broken_phase_fields(L + n, n, L)
    Bt32, B = factor(L, L)
    r = run_kernel(phi, L, Bt32, precision=precision)
    z = gpu_normals(5, 1, 3, 2, n, d)
    zr = oprec.round_operand(z, precision)
    Br = oprec.round_operand(B, precision)
    want = phi.astype(np.float64) + zr @ Br.T
    tol = product_tolerance(zr, Br, want)
    err = np.abs(r["prop"] - want)
    say("max err / tol", (err / tol).max())
    assert np.all(err <= tol)


def test_proposal_uses_oracle_stream_fp32():
    L, n = 8, 400
    phi = synth.broken_phase_fields(1, n, L)
    Bt32, B = factor(L, 2)
    r = run_kernel(phi, L, Bt32, seed=9, run=0, level=12, step0=19)
    want = osmc.propose(phi.astype(np.float64), B, 9, 0, 12, 19, np.arange(n), "fp64")
    z = orng.normals(9, 0, 12, 19, orng.PROPOSE, np.arange(n), L * L)
    tol = product_tolerance(z, B, want) + 4e-6 * (np.abs(z) @ np.abs(B).T)
    assert np.all(np.abs(r["prop"] - want) <= tol)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("L", [4, 8, 16, 18, 32])
def test_increment_is_odd_bitwise(precision, L):
    n = 64
    zero = np.zeros((n, L * L), dtype=np.float32)
    Bt32, _ = factor(L, 7)
    up = run_kernel(zero, L, Bt32, zsign=1.0, precision=precision)["prop"]
    dn = run_kernel(zero, L, Bt32, zsign=-1.0, precision=precision)["prop"]
    assert np.array_equal(dn, -up)
    assert np.any(up != 0)


TILES = [(32, 64, 256), (64, 64, 256), (128, 64, 256), (128, 128, 256), (128, 128, 512)]


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("L,n", [(17, 300), (24, 131)])
def test_every_product_tile(tile, precision, L, n):
    """Each tile of the three-pass product, pinned: the product against the
    float64 product of the same rounded operands, and bitwise oddness."""
    d = L * L
    say("tile", tile, precision, L, n)
    P.phi4_set_tile(n, d, precision, *tile)
    assert P.phi4_tile_choice(n, d, precision) == tile
    phi = synth.broken_phase_fields(L + n + 1, n, L)
    Bt32, B = factor(L, L + 1)
    r = run_kernel(phi, L, Bt32, precision=precision)
    z = gpu_normals(5, 1, 3, 2, n, d)
    zr = oprec.round_operand(z, precision)
    Br = oprec.round_operand(B, precision)
    want = phi.astype(np.float64) + zr @ Br.T
    assert np.all(np.abs(r["prop"] - want) <= product_tolerance(zr, Br, want))
    zero = np.zeros((n, d), dtype=np.float32)
    up = run_kernel(zero, L, Bt32, zsign=1.0, precision=precision)["prop"]
    dn = run_kernel(zero, L, Bt32, zsign=-1.0, precision=precision)["prop"]
    assert np.array_equal(dn, -up)


def test_set_tile_rejects_unknown_tiles():
    with pytest.raises(P.Phi4Error):
        P.phi4_set_tile(100, 289, "fp32", 48, 64)


def oracle_tempered(phi, prop, beta, L, seed, run, level, step, rows, m2=-4.0, lam=8.0):
    la = osmc.tempered_log_alpha(phi.astype(np.float64), prop.astype(np.float64), beta, L, m2, lam)
    lu = np.log(orng.accept_uniforms(seed, run, level, step, rows))
    return lu < la, la - lu


@pytest.mark.parametrize("L,n,beta", [(4, 256, 0.0), (8, 4096, 0.3), (8, 1000, 1.0),
                                      (10, 333, 0.7), (16, 2000, 0.5), (17, 300, 0.5),
                                      (18, 300, 0.5), (22, 203, 0.5), (32, 200, 0.5)])
def test_tempered_decisions(L, n, beta):
    say("tempered", L, n, beta)
    phi = synth.broken_phase_fields(n, n, L)
    Bt32, _ = factor(L, 3, scale=0.3)
    r = run_kernel(phi, L, Bt32, beta=beta)
    dec, margin = oracle_tempered(phi, r["prop"], beta, L, 5, 1, 3, 2, np.arange(n))
    bad = np.flatnonzero(dec != r["flags"])
    say("accepted", dec.mean(), "disagreements", len(bad), "margins", margin[bad])
    assert len(bad) <= max(1, int(1e-4 * n))
    assert np.all(np.abs(margin[bad]) < 1e-3)
    # accepted rows carry the proposal, the others the input, bitwise
    want = np.where(r["flags"][:, None], r["prop"], phi)
    assert np.array_equal(r["dst"], want)
    scale = oact.abs_site_sum(want.astype(np.float64), L, -4.0, 8.0)
    S64 = oact.action(want.astype(np.float64), L, -4.0, 8.0)
    assert np.all(np.abs(r["S"] - S64) <= 1e-5 * scale)
    np.testing.assert_allclose(r["absM"], np.abs(want.astype(np.float64).mean(1)), rtol=1e-5,
                               atol=1e-7)
    assert r["acc"] == int(r["flags"].sum())


@pytest.mark.parametrize("L,n", [(8, 3000), (17, 400), (22, 150), (32, 150)])
def test_constrained_decisions(L, n):
    pv = 4.0
    phi = synth.broken_phase_fields(77, n, L, v=0.2, noise=0.5)
    S0 = oact.action(phi.astype(np.float64), L, -4.0, 8.0)
    s_star = float(np.float32(np.median(S0)))
    Bt32, _ = factor(L, 5, scale=0.2)
    r = run_kernel(phi, L, Bt32, kind=1, s_star=s_star, prior_var=pv)
    prop = r["prop"].astype(np.float64)
    Sp = oact.action(prop, L, -4.0, 8.0)
    la = -(oact.u0(prop) - oact.u0(phi.astype(np.float64))) / pv
    lu = np.log(orng.accept_uniforms(5, 1, 3, 2, np.arange(n)))
    dec = (Sp < s_star) & (lu < la)
    bad = np.flatnonzero(dec != r["flags"])
    say("constrained accepted", dec.mean(), "disagreements", len(bad))
    assert len(bad) <= max(1, int(1e-4 * n))
    want = np.where(r["flags"][:, None], r["prop"], phi)
    assert np.array_equal(r["dst"], want)


@pytest.mark.parametrize("L", [8, 17, 24])
def test_row_list_in_place(L):
    n = 600
    phi = synth.broken_phase_fields(3, n, L)
    rows = synth.rng(4).choice(n, 250, replace=False).astype(np.int32)
    Bt32, B = factor(L, 8)
    r = run_kernel(phi, L, Bt32, rows=rows, inplace=True, beta=0.4)
    untouched = np.setdiff1d(np.arange(n), rows)
    assert np.array_equal(r["dst"][untouched], phi[untouched])
    z = gpu_normals(5, 1, 3, 2, len(rows), L * L, rows=rows)
    want = phi[rows].astype(np.float64) + z @ B.T
    assert np.all(np.abs(r["prop"] - want) <= product_tolerance(z, B, want))
    dec, _ = oracle_tempered(phi[rows], r["prop"], 0.4, L, 5, 1, 3, 2, rows)
    assert (dec != r["flags"]).sum() <= 1


@pytest.mark.parametrize("L,n,steps", [(4, 256, 10), (8, 2048, 20), (16, 512, 40),
                                       (17, 200, 5), (32, 128, 5)])
def test_multi_step_sweep_tracks_oracle(L, n, steps):
    """n fused steps vs the oracle stepping the same streams in float64."""
    say("sweep", L, n, steps)
    beta = 0.5
    phi = synth.broken_phase_fields(L * 100 + n, n, L)
    Bt32, B = factor(L, 9, scale=0.4)
    r = run_kernel(phi, L, Bt32, beta=beta, step0=0, n_steps=steps, level=6)
    ph = phi.astype(np.float64)
    S = oact.action(ph, L, -4.0, 8.0)
    n_acc = 0
    for s in range(steps):
        ph, S, acc = osmc.rwmh_step(ph, S, B, beta, L, -4.0, 8.0, 5, 1, 6, s)
        n_acc += int(acc.sum())
    close = np.all(np.abs(r["dst"] - ph) <= 1e-4 * (1 + np.abs(ph)), axis=1)
    say("rows tracking", close.mean(), "acc gpu", r["acc"], "oracle", n_acc)
    assert close.mean() >= 0.995
    assert abs(r["acc"] - n_acc) <= max(3, 0.002 * n_acc)
    scale = oact.abs_site_sum(r["dst"].astype(np.float64), L, -4.0, 8.0)
    assert np.all(np.abs(r["S"] - oact.action(r["dst"].astype(np.float64), L, -4.0, 8.0))
                  <= 1e-5 * scale)


@pytest.mark.parametrize("L", [8, 18])
def test_empty_and_zero_steps(L):
    phi = synth.fields(1, 40, L)
    Bt32, _ = factor(L, 1)
    r = run_kernel(phi, L, Bt32, n_steps=0)
    assert np.array_equal(r["dst"], phi) and r["acc"] == 0
    S64 = oact.action(phi.astype(np.float64), L, -4.0, 8.0)
    assert np.all(np.abs(r["S"] - S64) <= 1e-5 * oact.abs_site_sum(phi.astype(np.float64), L, -4.0, 8.0))
    r0 = run_kernel(phi[:0], L, Bt32)
    assert r0["dst"].shape == (0, L * L)
