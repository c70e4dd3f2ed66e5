#!/usr/bin/env python3
"""Throughput of adaptive tempered SMC-RW on 2D lattice phi^4 on one MI355X.

Workload (one step = one complete SMC run from beta = 0 to beta = 1):
L = 8 (d = 64 sites), N = 4096 particles, m0^2 = -4, lambda = 8, target ESS
N/2, 20 covariance-preconditioned random-walk Metropolis steps per tempering
level, float32 particles and proposal product, float64 reweighting / log Z /
Cholesky.  Each timed step restarts the run with its own Philox seed; all
inputs are synthetic draws of the sampler itself.

metric: particle-updates/s = N * n_steps * levels summed over the timed runs
divided by the wall time (one particle-update = one proposal plus
accept/reject of one particle's whole field; site-updates/s = that * d).

Also reported: the fused mutation kernel against its VALU roofline (HIP
events around every launch inside the timed region), the same workload with
the bfloat16 proposal product, |log Z - oracle| at seed 0 and the float64 CPU
oracle timed on the host (cpu_baseline).
"""

import argparse
import json
import math
import os
import sys
import time

WORKLOAD = dict(L=8, N=4096, m2=-4.0, lam=8.0, ess_frac=0.5, n_steps=20)

# Issue slots per site-update of the fused mutation kernel (VALU, per lane;
# full-rate op = 1 slot, quarter-rate transcendental / 32x32->64 multiply = 4):
#  Philox4x32-10: 10 rounds x (2 wide multiplies x 4 + 4 xor) / 4 normals = 30
#  Box-Muller:    (2 cvt + 2 fma + log 4 + mul + sqrt 4 + sin 4 + cos 4 + 2 mul) / 2 = 11.5
#  stencil, dS, dU0, accept and state update:                                 22
SLOTS_PER_SITE = 30.0 + 11.5 + 22.0
# VALU issue rate of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK = 256 * 4 * 16 * 2.4e9

# HBM bytes per launch of the fused sweep at this workload, from two rocprofv3
# counter runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0: the factors that make a
# 256 MiB device-to-device copy read and write 256 MiB on the same counters),
# valid only for the kernel sources they were taken on.
TRAFFIC = dict(bytes_per_launch=(522.71 * 1.99980 + 1072.0) * 1024,
               sources={"k_mutate.hip": "dc7ad60baebd00fc99def8042166cfc5d8093c1b793440617573e725636d07a0",
                        "common.hpp": "20b4425db3d352bda5372818ee91d001ee78f716f53557a5c19283103346c47b"})


def traffic_per_launch():
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2511_15196_amd", "csrc")
    for name, digest in TRAFFIC["sources"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return TRAFFIC["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the free-theory check and the L=16 SMC / L=32 NS workloads")
    ap.add_argument("--batch-levels", type=int, default=3,
                    help="levels of the 64-run batched workload (0: skip it; large values "
                         "run every run to beta = 1)")
    ap.add_argument("--only-extra", action="store_true",
                    help="run only the extra workloads and print them (profiling aid)")
    ap.add_argument("--extra-match", default="", metavar="SUBSTR",
                    help="with --only-extra: run only the extra workloads whose name contains SUBSTR")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="MIB",
                    help="only copy MIB mebibytes device-to-device with torch and exit "
                         "(calibrates the HBM byte counters of a profiler run)")
    return ap.parse_args()


def timed_runs(P, torch, precision, steps, warmup, seed0=0):
    w = WORKLOAD
    smc = P.SMC(w["L"], w["N"], w["m2"], w["lam"], ess_frac=w["ess_frac"],
                n_steps=w["n_steps"], seed=seed0, precision=precision)
    for i in range(warmup):
        smc.restart(100000 + i)
        smc.run()
    P.phi4_kernel_time(smc.h)                 # drop warm-up records
    P.phi4_set_timing(smc.h, True)
    levels, logzs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        smc.restart(seed0 + i)
        rc, lv = smc.run()
        levels.append(lv)
        if i == 0:
            logzs.append(smc.logz())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = P.phi4_kernel_time(smc.h)
    P.phi4_set_timing(smc.h, False)
    smc.close()
    pu = sum(levels) * w["N"] * w["n_steps"]
    return dict(wall=wall, levels=levels, pu=pu, kernel_ms=kms, launches=launches,
                logz_seed0=logzs[0])


def cpu_baseline():
    """The float64 oracle, one thread, one full run of the workload (seed 0)."""
    from threadpoolctl import threadpool_limits
    from oracle import smc as osmc
    w = WORKLOAD
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = osmc.smc_run(w["L"], w["m2"], w["lam"], w["N"], w["ess_frac"], w["n_steps"], seed=0)
        dt = time.perf_counter() - t0
    pu = r["n_levels"] * w["N"] * w["n_steps"]
    return dict(value=pu / dt, unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"one full SMC run of the workload, seed 0, {r['n_levels']} levels, "
                       f"{dt:.1f} s, float64 numpy on 1 host thread",
                logz=r["logz"])


def free_log_z(L, m2):
    """Exact log Z of the free theory (lambda = 0) under the N(0, I) reference:
    -1/2 sum_k log(1 + m2 + lambda_k), lambda_k the periodic lattice-Laplacian
    eigenvalues 4 sin^2(pi k0 / L) + 4 sin^2(pi k1 / L)."""
    t = 0.0
    for k0 in range(L):
        for k1 in range(L):
            lk = 4 * math.sin(math.pi * k0 / L) ** 2 + 4 * math.sin(math.pi * k1 / L) ** 2
            t += math.log(1.0 + m2 + lk)
    return -0.5 * t


def smc_workload(P, torch, L, N, m2, lam, n_steps, precision, seed=0, kernel="rw"):
    """One warm-up run and one timed full SMC run (seed `seed`)."""
    smc = P.SMC(L, N, m2, lam, ess_frac=0.5, n_steps=n_steps, seed=seed, precision=precision,
                kernel=kernel)
    smc.restart(seed + 1000)
    smc.run()
    smc.restart(seed)
    P.phi4_kernel_time(smc.h)
    P.phi4_set_timing(smc.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, lv = smc.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = P.phi4_kernel_time(smc.h)
    obs = smc.observables()
    out = dict(value=lv * N * n_steps / wall, levels=lv, ms_per_run=wall * 1e3,
               logz=smc.logz(), mean_abs_m=obs["mean_abs_m"], acc=obs["acc"],
               sweep_ms_per_level=kms / max(launches, 1))
    smc.close()
    return out


def ns_workload(P, torch, L, n, k, n_steps, precision, iters, warm=2, seed=0, kernel="rw"):
    """`iters` timed nested-sampling iterations after `warm` untimed ones."""
    ns = P.NS(L, n, k, n_steps, -4.0, 8.0, prior_var=4.0, term_frac=1e-3, seed=seed,
              precision=precision, kernel=kernel)
    for _ in range(warm):
        P.ns_step(ns.h, sync=False)
    P.phi4_kernel_time(ns.h)
    P.phi4_set_timing(ns.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        P.ns_step(ns.h, sync=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = P.phi4_kernel_time(ns.h)
    d = L * L
    sweep_s = kms * 1e-3 / max(launches, 1)
    out = dict(value=iters * k * n_steps / wall, ms_per_iter=wall / iters * 1e3,
               sweep_ms=sweep_s * 1e3,
               proposal_tflops_in_sweep=k * n_steps * d * (d + 1) / sweep_s / 1e12)
    ns.close()
    return out


def batch_workload(P, torch, max_levels, n=8192, n_steps=20):
    """64 independent SMC runs advanced together: L = (8, 16, 32, 64)[r mod 4],
    (m2, lambda) = grid[(r div 4) mod 6] over m2 in (-4, -2, -1) x lambda in
    (4, 8), float32 proposal products for runs 0-23 and 48-63, bfloat16 for
    24-47; N = 8192 each, Philox key (seed 0, run r)."""
    grid = [(m2, lam) for m2 in (-4.0, -2.0, -1.0) for lam in (4.0, 8.0)]
    cfg = []
    for r in range(64):
        m2, lam = grid[(r // 4) % 6]
        cfg.append(((8, 16, 32, 64)[r % 4], m2, lam, "fp32" if (r // 24) % 2 == 0 else "bf16"))
    # time the proposal-product tiles of the large shapes outside the timed region
    for L in (32, 64):
        for prec in ("fp32", "bf16"):
            t = P.SMC(L, n, -4.0, 8.0, ess_frac=0.5, n_steps=1, seed=1, precision=prec)
            P.smc_reweight_resample(t.h)
            P.smc_mutate(t.h)
            t.close()
    progress("batch: tiles timed")
    runs = [P.SMC(L, n, m2, lam, ess_frac=0.5, n_steps=n_steps, seed=0, run=r, precision=prec)
            for r, (L, m2, lam, prec) in enumerate(cfg)]
    progress("batch: 64 runs initialised")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, levels = P.smc_batch_run([s.h for s in runs], max_levels=max_levels)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pu = sum(levels) * n * n_steps
    su = sum(lv * n * n_steps * L * L for lv, (L, _, _, _) in zip(levels, cfg))
    per_run = []
    for s, lv, (L, m2, lam, prec) in zip(runs, levels, cfg):
        per_run.append(dict(L=L, m2=m2, lam=lam, precision=prec, levels=lv,
                            beta=s.observables()["beta_or_logX"], logz=s.logz(),
                            mean_abs_m=s.observables()["mean_abs_m"]))
        s.close()
    tiles = {f"L{L}_{prec}": P.phi4_tile_choice(n, L * L, prec)
             for L in (32, 64) for prec in ("fp32", "bf16")}
    return dict(value=pu / wall, site_updates_per_s=su / wall, wall_s=wall,
                all_finished=rc == P.PHI4_DONE, max_levels=max_levels, n=n, n_steps=n_steps,
                gemm_tile_rows=tiles, runs=per_run)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The paper's SMC-RW runs on one NVIDIA L4 (Table 2): wall-clock seconds and
# log Z at m0^2 = -4, lambda = 1, N = 5000, 3V steps per level, ESS 0.9.
PAPER_SMC_RW_L4 = {10: (6.7, -65.2), 15: (21.5, -146.4), 18: (46.0, -209.9)}


def paper_point(P, torch, sizes=(10, 15, 18), seed=0):
    """SMC-RW at the paper's own settings, timed end to end on this GPU."""
    out = {}
    for L in sizes:
        d = L * L
        warm = P.SMC(L, 5000, -4.0, 1.0, ess_frac=0.9, n_steps=1, seed=seed + 1000)
        P.smc_reweight_resample(warm.h)
        P.smc_mutate(warm.h)
        warm.close()
        smc = P.SMC(L, 5000, -4.0, 1.0, ess_frac=0.9, n_steps=3 * d, seed=seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, lv = smc.run()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ref_s, ref_z = PAPER_SMC_RW_L4[L]
        out[f"L{L}"] = dict(seconds=wall, levels=lv, logz=smc.logz(),
                            mean_abs_m=smc.observables()["mean_abs_m"],
                            value=lv * 5000 * 3 * d / wall,
                            paper_L4_seconds=ref_s, paper_L4_logz=ref_z)
        smc.close()
        progress(f"paper point L={L} done")
    return out


def extra_workloads(P, torch, match=""):
    """Free-theory check of the main workload, SMC-RW, SMC-IRMH and SMC-HMC at
    L = 8 .. 32, NS at L = 32 and the paper's own point; `match` keeps the
    names containing it."""
    ex = {}

    def want(name):
        return match in name

    if want("free_theory_L8"):
        progress("free-theory check")
        fz = smc_workload(P, torch, 8, 4096, 1.0, 0.0, 20, "fp32")
        exact = free_log_z(8, 1.0)
        ex["free_theory_L8"] = dict(logz=fz["logz"], exact=exact, dlogz=fz["logz"] - exact,
                                    levels=fz["levels"], note="m2=1, lambda=0, N=4096, 20 steps/"
                                    "level; the gap is the method's finite-mixing bias, shared by "
                                    "the oracle")
    for lam in (5.0, 8.0):
        for prec in ("fp32", "bf16"):
            name = f"smc_L16_N16384_lam{lam:g}_{prec}"
            if want(name):
                ex[name] = smc_workload(P, torch, 16, 16384, -4.0, lam, 20, prec)
                progress(f"SMC L=16 lambda={lam:g} {prec} done")
    for L in (8, 16, 32):
        name = f"smc_irmh_L{L}_N16384_lam8_fp32"
        if want(name):
            ex[name] = smc_workload(P, torch, L, 16384, -4.0, 8.0, 20, "fp32", kernel="irmh")
            progress(f"SMC-IRMH L={L} done")
    for L in (8, 16, 32):
        name = f"smc_hmc_L{L}_N16384_lam8_fp32"
        if want(name):
            r = smc_workload(P, torch, L, 16384, -4.0, 8.0, 5, "fp32", kernel="hmc")
            # one particle-update = one 20-step trajectory; a leapfrog step evaluates
            # the gradient at every site once
            r["gradient_site_evals_per_s"] = r["value"] * 20 * L * L
            ex[name] = r
            progress(f"SMC-HMC L={L} done")
    for prec in ("fp32", "bf16"):
        name = f"ns_L32_n4096_k2048_{prec}"
        if want(name):
            ex[name] = ns_workload(P, torch, 32, 4096, 2048, 40, prec, 8)
            progress(f"NS L=32 {prec} done")
    for L in (16, 32):
        name = f"ns_slice_L{L}_n4096_k2048_fp32"
        if want(name):
            # one particle-update = one slice move of one refilled point
            ex[name] = ns_workload(P, torch, L, 4096, 2048, 5, "fp32", 8, kernel="slice")
            progress(f"NS slice L={L} done")
    if want("paper_point_smc_rw"):
        ex["paper_point_smc_rw"] = paper_point(P, torch)
    return ex


def product_tiles(P, torch, L=64, N=8192, steps=5):
    """The proposal product at one large shape with every tile pinned in turn:
    a 5-step sweep (normals, product, accept per step) after one level, per
    precision and tile, timed with HIP events (profiling aid)."""
    d = L * L
    out = {}
    for prec in ("bf16", "fp32"):
        for tile in [(32, 64, 256), (64, 64, 256), (128, 64, 256), (128, 128, 256), (128, 128, 512)]:
            P.phi4_set_tile(N, d, prec, *tile)
            s = P.SMC(L, N, -4.0, 8.0, ess_frac=0.5, n_steps=steps, seed=0, precision=prec)
            P.smc_reweight_resample(s.h)
            torch.cuda.synchronize()
            P.phi4_set_timing(s.h, True)
            P.smc_mutate(s.h)
            torch.cuda.synchronize()
            ms, _ = P.phi4_kernel_time(s.h)
            out[f"{prec}_{tile[0]}x{tile[1]}x{tile[2]}"] = dict(sweep_ms=ms, steps=steps)
            s.close()
    return out


def copy_probe(torch, mib):
    n = int(mib * (1 << 20)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "launches": 3}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent runs shard across GPUs without communication; see the design "
              "notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2511_15196_amd as P

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe > 0:
        copy_probe(torch, args.copy_probe)
        return
    if args.only_extra:
        ex = extra_workloads(P, torch, args.extra_match)
        if args.extra_match and args.extra_match in "product_tiles_L64_N8192":
            ex["product_tiles_L64_N8192"] = product_tiles(P, torch)
        if args.batch_levels > 0 and args.extra_match in "batch64":
            ex["batch64"] = batch_workload(P, torch, args.batch_levels)
        print(json.dumps({"workloads": ex}), flush=True)
        return
    w = WORKLOAD
    d = w["L"] ** 2
    r = timed_runs(P, torch, args.precision, args.steps, args.warmup)
    value = r["pu"] / r["wall"]
    k_avg = r["kernel_ms"] / max(r["launches"], 1) * 1e-3          # s per launch
    pu_launch = w["N"] * w["n_steps"]
    achieved = pu_launch * d * SLOTS_PER_SITE / k_avg
    mfma_tflops = pu_launch * d * (d + 1) / k_avg / 1e12
    line = {
        "metric": "particle-updates/s",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": "adaptive tempered SMC-RW, 2D phi^4 L=8 (d=64), N=4096, "
                               "m2=-4, lambda=8, ESS N/2, 20 RW-MH steps/level",
                   "L": w["L"], "N": w["N"], "n_steps": w["n_steps"], "ess_frac": w["ess_frac"],
                   "precision": args.precision, "parallelism": "single GPU"},
        "site_updates_per_s": value * d,
        "levels_mean": sum(r["levels"]) / len(r["levels"]),
        "logz_seed0": r["logz_seed0"],
        "mutate_kernel_us": k_avg * 1e6,
        "mutate_kernel_share": r["kernel_ms"] * 1e-3 / r["wall"],
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK, "traffic": traffic_per_launch(),
                     "kernel": "mutate_kernel<DP=64,W=4,fp32>",
                     "mfma_tflops": mfma_tflops},
    }
    if not args.no_bf16 and args.precision == "fp32":
        rb = timed_runs(P, torch, "bf16", max(2, args.steps // 2), 1)
        line["bf16"] = {"value": rb["pu"] / rb["wall"], "logz_seed0": rb["logz_seed0"],
                        "mutate_kernel_us": rb["kernel_ms"] / max(rb["launches"], 1) * 1e3}
    if not args.no_extra and args.precision == "fp32":
        line["workloads"] = extra_workloads(P, torch)
        if args.batch_levels > 0:
            line["workloads"]["batch64"] = batch_workload(P, torch, args.batch_levels)
    if not args.no_cpu_baseline:
        cb = cpu_baseline()
        line["dlogz_vs_oracle_seed0"] = abs(r["logz_seed0"] - cb.pop("logz"))
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
