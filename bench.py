"""Benchmark: cell-updates per second per SSP-RK3 stage of the PP Active
Flux MHD scheme on one MI355X (FP64), Orszag-Tang vortex on a 512x512
periodic grid (synthetic initial data; inputs resident in HBM before the
timed region).

python bench.py [--steps K] [--warmup W] [--workload orszag_tang_512|blast_lowbeta_1024|alfven_32]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell per stage (FP64 storage, 4 DoF sets x 8 variables):
# read U^n and U^(k) (256 B each; one array at k = 0), write U^(k+1) (256 B)
BYTES_PER_CELL_STAGE = (512 + 768 + 768) / 3.0


def cpu_baseline(prob, u0, budget_s=12.0):
    """The CPU oracle timed on a bounded sample of the same workload."""
    from oracle import oracle as orc
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    dt = orc.dt(prob, u0, nthreads=threads)
    t0 = time.perf_counter()
    n = 0
    u = u0
    while True:
        u = orc.stage(prob, 0, u0, u0, dt, nthreads=threads)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": prob.nx * prob.ny * n / el, "unit": "cell-updates/s per RK stage", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} forward-Euler stages of {prob.name} {prob.nx}x{prob.ny} from the initial data, "
                      f"{el:.1f} s, FP64 C++ oracle with OpenMP"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="orszag_tang_512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2506_04857_amd import af_mhd as af
    from paper_2506_04857_amd import inputs as I

    prob = I.CONFIGS[args.workload]()
    u0 = I.sample(prob)
    ctx = af.Context(prob)
    u = af.to_device(u0)
    stream = ctx.stream
    for _ in range(args.warmup):
        ctx.af_mhd_step(u)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.af_mhd_step(u)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    st = ctx.af_mhd_stats(u)
    cells = prob.nx * prob.ny
    stages = 3 * args.steps
    t_stage = ms * 1e-3 / stages
    value = cells / t_stage
    achieved = BYTES_PER_CELL_STAGE * cells / t_stage / 1e9
    out = {
        "metric": "cell-updates/s per RK stage (FP64), %HBM peak",
        "value": value,
        "unit": "cell-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{prob.name} {prob.nx}x{prob.ny}", "nx": prob.nx, "ny": prob.ny,
                   "cells": cells, "precision": "fp64", "cfl": prob.cfl, "kappa": prob.kappa},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "admissible": bool(st["admissible"]),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, u0)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
