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


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
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
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK, "traffic": None,
                     "kernel": "mutate_kernel<DP=64,W=4,fp32>",
                     "mfma_tflops": mfma_tflops},
    }
    if not args.no_bf16 and args.precision == "fp32":
        rb = timed_runs(P, torch, "bf16", max(2, args.steps // 2), 1)
        line["bf16"] = {"value": rb["pu"] / rb["wall"], "logz_seed0": rb["logz_seed0"],
                        "mutate_kernel_us": rb["kernel_ms"] / max(rb["launches"], 1) * 1e3}
    if not args.no_cpu_baseline:
        cb = cpu_baseline()
        line["dlogz_vs_oracle_seed0"] = abs(r["logz_seed0"] - cb.pop("logz"))
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
