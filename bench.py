"""Benchmark: cell-updates per second per SSP-RK3 stage of the PP Active
Flux MHD scheme on one MI355X (FP64), low-beta blast on a 1024x1024 outflow
grid (synthetic initial data; inputs resident in HBM before the timed
region; the state sets, 1.07 GB per step with U^n, U^(k) and the output,
are past the 256 MB Infinity Cache).

python bench.py [--steps K] [--warmup W] [--workload blast_lowbeta_1024|orszag_tang_512|alfven_32]
Prints one JSON line.

roofline: the whole stage against HBM -- the stage's algorithmic bytes
(682.7 B per cell, mean over the three stages) over the average device time
of one stage's kernels (point kernel + cell kernel + a third of the step's
time-step reduction), from HIP events on the launch stream.

Also measured (objects of the same line): the FP32-bulk stage, the
Orszag-Tang 512^2 workload, the batched ensemble, the adjoint workload
(adjoint/forward time, finite-difference and oracle-reference checks of the
gradient) and the CPU oracle baseline (single-threaded and on all host
cores).

python bench.py --copy-calibration MIB
runs a plain device-to-device copy of MIB MiB three times (the known-size
kernel against which rocprofv3's FETCH_SIZE / WRITE_SIZE are scaled) and exits.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK stage (FP64 vs FP32-bulk), %HBM peak; adjoint/fwd time"
UNIT = "cell-updates/s per RK stage"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per cell (FP64 storage; 4 DoF sets x 8 variables,
# 64 B per set), averaged over the three stages (a_k = 0 at k = 0, so U^n
# is not read there):
#   whole stage: read U^(k) 256, read U^n 256 (k >= 1), write 256
BYTES_PER_CELL_STAGE = (512 + 768 + 768) / 3.0
#   cell-average kernel: read U^(k) (all four sets) 256, read A^n 64 (k >= 1),
#   write A 64
BYTES_PER_CELL_CELLS = 256 + 64 * 2.0 / 3.0 + 64
#   point kernel: read U^(k) 256, read X^n, Y^n, V^n 192 (k >= 1), write 192
BYTES_PER_CELL_POINTS = 256 + 192 * 2.0 / 3.0 + 192

# rocprofv3 summaries of the stage kernels per workload (committed under
# profiles/): HBM traffic (FETCH_SIZE, WRITE_SIZE) and VALU instruction counts
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILES = {"blast_lowbeta_1024": "k_points_k_cells_blast_lowbeta_1024_hbm_traffic.txt",
                 "orszag_tang_512": "k_points_k_cells_orszag_tang_512_hbm_traffic.txt"}
VALU_FILES = {"blast_lowbeta_1024": "k_points_k_cells_blast_lowbeta_1024_valu.txt",
              "orszag_tang_512": "k_points_k_cells_orszag_tang_512_valu.txt"}
CUS, CLOCK_HZ = 256, 2.4e9  # MI355X: one wave-instruction issued per CU per cycle at most


# The sources the stage kernels k_points / k_cells are built from (the
# traffic measurement is theirs; the batch and adjoint sources do not enter).
STAGE_SOURCES = [os.path.join(ROOT, "paper_2506_04857_amd", "csrc", f)
                 for f in ("af_stage.hip", "af_device.h", "af_tiles.h")] + [os.path.join(ROOT, "include", "af_mhd.h")]


def source_hash() -> str:
    """SHA-256 over the sources of the stage kernels."""
    h = hashlib.sha256()
    for path in STAGE_SOURCES:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode() + b"\0" + fh.read())
    return h.hexdigest()


def profile_values(fname: str):
    """key: value pairs of a committed profile summary, or None when it is
    missing or was taken from a different kernel source."""
    path = os.path.join(PROFILES, fname)
    if not fname or not os.path.isfile(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    return kv


def stage_mean(kv, prefix: str, kernel: str):
    """Per-launch value of a kernel averaged over the three stages of a step.
    The stage kernels are instantiated twice: `<double, false>` runs stages
    0 and 1, `<double, true>` the last stage, which also reduces the next
    time step's wave speeds; a kernel with one instantiation is taken as is."""
    if kv is None:
        return None
    try:
        if kernel.endswith("<double>"):
            base = kernel[:-len("<double>")]
            a = float(kv[f"{prefix}.{base}<double, false>"])
            b = float(kv[f"{prefix}.{base}<double, true>"])
            return (2.0 * a + b) / 3.0
        return float(kv[f"{prefix}.{kernel}"])
    except (KeyError, ValueError):
        return None


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of the kernel (mean over a step's stages) from
    the committed rocprofv3 counter summary, or None."""
    return stage_mean(profile_values(TRAFFIC_FILES.get(workload, "")), "traffic_bytes_per_launch", kernel)


def measured_valu(workload: str, kernel: str):
    """VALU wave-instructions per launch of the kernel (mean over a step's
    stages) from the committed SQ counter summary, or None."""
    return stage_mean(profile_values(VALU_FILES.get(workload, "")), "valu_insts_per_launch", kernel)


def cpu_baseline(prob, u0, budget_s=10.0):
    """The CPU oracle timed on a bounded sample of the same workload:
    forward-Euler stages from the initial data, single-threaded and with
    OpenMP over rows on all the host cores it is given."""
    from oracle import oracle as orc
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()

    def rate(nthreads):
        dt = orc.dt(prob, u0, nthreads=nthreads)
        t0 = time.perf_counter()
        n = 0
        while True:
            orc.stage(prob, 0, u0, u0, dt, nthreads=nthreads)
            n += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        el = time.perf_counter() - t0
        return prob.nx * prob.ny * n / el, n, el

    v_all, n_all, el_all = rate(threads)
    v_one, n_one, el_one = rate(1)
    return {"value": v_all, "unit": UNIT, "cores": threads, "kind": "oracle",
            "single_thread": {"value": v_one, "unit": UNIT, "cores": 1},
            "sample": f"forward-Euler stages of {prob.name} {prob.nx}x{prob.ny} from the initial data (FP64 C++ "
                      f"oracle): {n_all} stages in {el_all:.1f} s on {threads} threads (OpenMP over rows), "
                      f"{n_one} in {el_one:.1f} s on one"}


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "launches": 3}))


def stream_copy_gbs(af, mib: int = 1024, reps: int = 20) -> dict:
    """Bandwidth of the library's own stream-copy kernel (read + write bytes
    per second) on a mib MiB buffer, HIP events on its stream."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    for _ in range(3):
        af.stream_copy(src, dst, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        af.stream_copy(src, dst, s)
    e1.record(s)
    torch.cuda.synchronize()
    assert bool(torch.equal(src, dst))
    ms = e0.elapsed_time(e1) / reps
    return {"gbs": 2 * n * 8 / (ms * 1e-3) / 1e9, "bytes": n * 8, "ms": ms}


def timed_steps(ctx, u, steps, stream):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        ctx.af_mhd_step(u)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


TILE_TABLE = os.path.join(ROOT, "paper_2506_04857_amd", "tiles_mi355x.txt")
MODE_NAMES = {0: "flat", 1: "persistent", 2: "fused"}


def batched(af, I, args):
    """The batched Orszag-Tang ensemble: 256 instances of sizes drawn from
    {64,96,128,192,256}^2 with perturbed fields, all stepped together (one
    hipGraph per step; cell tiles from the autotuned table; the launch mode
    the batch's tuner picks, and each of the three modes timed on the same
    batch), FP64 and FP32-bulk; against the same instances stepped one after
    another by single-grid contexts."""
    import shutil
    import tempfile

    import torch
    probs = I.batched_orszag_tang(256)
    u0s = [I.sample(p, gl=2) for p in probs]
    cells = sum(p.nx * p.ny for p in probs)
    table = os.path.join(tempfile.mkdtemp(), "tiles.txt")
    if os.path.exists(TILE_TABLE):
        shutil.copy(TILE_TABLE, table)
    res = {}
    for name, flags in (("fp64", 0), ("fp32", af.AF_FLAG_FP32_BULK)):
        states = [af.to_device(u) for u in u0s]
        b = af.Batch(probs, states, flags=flags, tune_table=table)
        for _ in range(args.warmup):
            b.step()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(b.stream)
        for _ in range(args.steps):
            b.step()
        ev1.record(b.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        tiles = {}
        for m in range(len(probs)):
            key = "%dx%d" % b.tile(m)
            tiles[key] = tiles.get(key, 0) + 1
        chosen = b.launch_mode()
        res[name] = {"value": cells * 3 * args.steps / (ms * 1e-3), "ms_per_step": ms / args.steps,
                     "mode": MODE_NAMES[chosen], "persistent": b.persistent(), "tiles": tiles}
        if name == "fp64":
            # every launch mode on the same batch (graph replays, 20 steps each)
            modes = {}
            for mode in (af.AF_BATCH_FLAT, af.AF_BATCH_PERSISTENT, af.AF_BATCH_FUSED):
                b.set_launch_mode(mode)
                for _ in range(2):
                    b.step()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(b.stream)
                for _ in range(20):
                    b.step()
                e1.record(b.stream)
                torch.cuda.synchronize()
                modes[MODE_NAMES[mode]] = {"value": cells * 3 * 20 / (e0.elapsed_time(e1) * 1e-3),
                                           "launches_per_stage": 1 if mode == af.AF_BATCH_FUSED else 2}
            res[name]["modes"] = modes
        b.close()
        del states
    # the same instances one after another, single-grid contexts, FP64
    nseq = max(1, min(args.steps, 20))
    ctxs = [af.Context(p) for p in probs]
    us = [af.to_device(u) for u in u0s]
    for c, u in zip(ctxs, us):
        c.af_mhd_step(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, u in zip(ctxs, us):
        for _ in range(nseq):
            c.af_mhd_step(u)
    torch.cuda.synchronize()
    seq = cells * 3 * nseq / (time.perf_counter() - t0)
    for c in ctxs:
        c.close()
    with open(table) as fh:
        tuned = [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]
    if args.save_tile_table:
        shutil.copy(table, args.save_tile_table)
    return {"value": res["fp64"]["value"], "unit": UNIT, "instances": len(probs), "cells": cells,
            "ms_per_step": res["fp64"]["ms_per_step"], "graph": True, "mode": res["fp64"]["mode"],
            "launches_per_stage": 1 if res["fp64"]["mode"] == "fused" else 2, "launches_per_step_dt": 2,
            "modes": res["fp64"]["modes"],
            "persistent": res["fp64"]["persistent"], "tiles": res["fp64"]["tiles"],
            "sequential_value": seq, "speedup_vs_sequential": res["fp64"]["value"] / seq,
            "fp32_bulk": res["fp32"], "fp32_speedup_vs_fp64": res["fp32"]["value"] / res["fp64"]["value"],
            "size_classes_tuned": len(tuned),
            "inputs": "256 periodic Orszag-Tang instances, nx, ny from {64,96,128,192,256}, fields x (1 + 0.05 z), "
                      "2x2 Gauss cell averages"}


ADJ_REFERENCE = os.path.join(ROOT, "tests", "golden", "adjoint_reference_alfven_perturbed_256.json")


def adjoint(af, I, args):
    """The adjoint workload: gradient of J = 1/2 sum (rho(T) - 1)^2 with
    respect to all 32 initial planes of the perturbed Alfven wave (256^2,
    kappa 1, 400 SSP-RK3 steps), the forward's tapes kept when they fit half
    the free device memory (else sqrt(n) checkpointing, every 20 steps), dt
    sequence frozen.  Reports adjoint/forward time, central differences
    (h = 1e-6) on 20 seeded directions and, when present, the FP64 CPU
    reference (tangent oracle) along 8 directions with the oracle's dts."""
    import numpy as np
    import torch

    prob = I.alfven_perturbed(256)
    nsteps, every = I.ADJOINT_STEPS, 20
    u0 = I.sample(prob)
    u0d = af.to_device(u0)

    def J_of(uT):
        return 0.5 * float(torch.sum((uT[0][0] - I.adjoint_objective_target(prob)) ** 2))

    def grad(dts=None):
        run = af.CheckpointedRun(prob, every=every)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        ev[0].record(run.ctx.stream)
        uT = run.forward(u0d, nsteps, dts=dts)
        ev[1].record(run.ctx.stream)
        lam = tuple(torch.zeros_like(t) for t in uT)
        lam[0][0].copy_(uT[0][0] - I.adjoint_objective_target(prob))
        g = run.backward(lam)
        ev[2].record(run.ctx.stream)
        torch.cuda.synchronize()
        used = run.dts.clone()
        kept = {"tape_bytes_per_stage": run.adj.tape_bytes,
                "kept_bytes": run.step_bytes() * nsteps if run.tapes_kept else 0}
        run.close()
        return af.to_host(g), used, ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), J_of(uT), kept

    def J_fixed(u, dts):
        run = af.CheckpointedRun(prob, every=nsteps, keep_tapes=False)
        uT = run.forward(af.to_device(u), nsteps, dts=dts)
        torch.cuda.synchronize()
        run.close()
        return J_of(uT)

    grad()  # warm-up (kernel loading, allocator)
    g, dts, fwd_ckpt_ms, bwd_ms, J, kept = grad()
    # the plain forward: 400 whole steps of the stage kernels, no checkpoints
    ctx = af.Context(prob, flags=af.AF_FLAG_FUSED_DT)
    u = af.to_device(u0)
    fwd_ms = timed_steps(ctx, u, nsteps, ctx.stream)
    ctx.close()
    # central differences on 20 seeded directions, same dt sequence
    h = 1e-6
    errs = []
    for v in I.adjoint_directions(prob, 20):
        got = sum(float(np.sum(a * b)) for a, b in zip(g, v))
        fd = (J_fixed(tuple(a + h * b for a, b in zip(u0, v)), dts)
              - J_fixed(tuple(a - h * b for a, b in zip(u0, v)), dts)) / (2 * h)
        errs.append(abs(got - fd) / abs(fd))
    out = {"workload": f"alfven_perturbed {prob.nx}x{prob.ny}, kappa {prob.kappa}, {nsteps} steps",
           "objective": "J = 1/2 sum (rho(T) - 1)^2, gradient w.r.t. all 32 initial planes",
           "forward_ms": fwd_ms, "forward_recording_ms": fwd_ckpt_ms, "backward_ms": bwd_ms,
           "adjoint_over_forward": (fwd_ckpt_ms + bwd_ms) / fwd_ms,
           "forward_mode": ("recording stage, every step's stage inputs and tapes kept: the backward sweeps "
                            "the forward's own tapes" if kept["kept_bytes"] else
                            "recording stage with a checkpoint every %d steps: the backward recomputes each "
                            "segment bit for bit" % every),
           "tape_bytes_per_stage": kept["tape_bytes_per_stage"], "kept_gb": kept["kept_bytes"] / 1e9, "J": J,
           "fd": {"directions": 20, "h": h, "max_rel": max(errs), "median_rel": float(np.median(errs))}}
    if os.path.exists(ADJ_REFERENCE):
        with open(ADJ_REFERENCE) as fh:
            ref = json.load(fh)
        g2, _, _, _, J2, _ = grad(dts=torch.tensor(ref["dts"], dtype=torch.float64, device="cuda"))
        rel = []
        for v, want in zip(I.adjoint_directions(prob, len(ref["dJ"])), ref["dJ"]):
            got = sum(float(np.sum(a * b)) for a, b in zip(g2, v))
            rel.append(abs(got - want) / abs(want))
        out["oracle_reference"] = {"directions": len(rel), "max_rel": max(rel), "median_rel": float(np.median(rel)),
                                   "J_rel": abs(J2 - ref["J"]) / ref["J"]}
    return out


def stage_run(af, prob, u0, args, flags):
    """Timed region: K whole steps (time step + three stages) after W
    warm-up steps, no timing events; then the same with per-kernel HIP
    events on the launch stream (AF_FLAG_KERNEL_TIMING) for the kernels'
    average launch durations.  The step's time step is the fused one
    (AF_FLAG_FUSED_DT: the last stage leaves the wave-speed maxima).
    Returns (ms for K steps, stats, final state, average us per launch)."""
    flags |= af.AF_FLAG_FUSED_DT
    ctx = af.Context(prob, flags=flags)
    u = af.to_device(u0)
    for _ in range(args.warmup):
        ctx.af_mhd_step(u)
    ms = timed_steps(ctx, u, args.steps, ctx.stream)
    st = ctx.af_mhd_stats(u)
    ctx.close()
    tctx = af.Context(prob, flags=flags | af.AF_FLAG_KERNEL_TIMING)
    v = af.to_device(u0)
    for _ in range(args.warmup):
        tctx.af_mhd_step(v)
    tctx.af_mhd_kernel_times(reset=True)
    timed_steps(tctx, v, args.steps, tctx.stream)
    kt = tctx.af_mhd_kernel_times()
    tctx.close()
    us = {"k_cells": 1e3 * kt["ms_cells"] / max(kt["n_cells"], 1),
          "k_points": 1e3 * kt["ms_points"] / max(kt["n_points"], 1),
          "dt": 1e3 * kt["ms_dt"] / max(kt["n_dt"], 1)}
    return ms, st, af.to_host(u), us


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="blast_lowbeta_1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-ensemble measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint measurement")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workloads (FP32-bulk, Orszag-Tang 512^2, graph replay, stream copy)")
    ap.add_argument("--adjoint-only", action="store_true", help="only the adjoint measurement (its JSON object)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched-ensemble measurement (its JSON object), e.g. for profiling it")
    ap.add_argument("--save-tile-table", default="", metavar="PATH",
                    help="write the cell-tile table the batch used (with new measurements) to PATH")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; multi-GPU runs are not supported "
                                   "(--gpus must be 1)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    from paper_2506_04857_amd import af_mhd as af
    from paper_2506_04857_amd import inputs as I

    if args.batch_only:
        print(json.dumps({"batched": batched(af, I, args)}))
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint(af, I, args)}))
        return

    prob = I.CONFIGS[args.workload]()
    u0 = I.sample(prob)
    cells = prob.nx * prob.ny
    stages = 3 * args.steps

    ms, st, u64, us = stage_run(af, prob, u0, args, 0)
    t_stage = ms * 1e-3 / stages
    value = cells / t_stage

    # roofline: the whole stage (both kernels and a third of the step's time
    # step) against HBM, by the stage's algorithmic bytes
    stage_bytes = BYTES_PER_CELL_STAGE * cells
    stage_us = us["k_points"] + us["k_cells"] + us["dt"] / 3.0
    achieved = stage_bytes / (stage_us * 1e-6) / 1e9
    per_kernel = {}
    for kname, bpc in (("k_points", BYTES_PER_CELL_POINTS), ("k_cells", BYTES_PER_CELL_CELLS)):
        a = bpc * cells / (us[kname] * 1e-6) / 1e9
        per_kernel[kname] = {"achieved": a, "frac": a / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": bpc * cells,
                             "avg_launch_us": us[kname],
                             "traffic": measured_traffic(args.workload, kname + "<double>")}
    parts = [measured_traffic(args.workload, k) for k in ("k_points<double>", "k_cells<double>", "k_dt_from_parts")]
    traffic = None if any(p is None for p in parts) else parts[0] + parts[1] + parts[2] / 3.0
    # VALU issue: wave-instructions per cell-stage against one per CU per cycle
    vparts = [measured_valu(args.workload, k) for k in ("k_points<double>", "k_cells<double>")]
    valu = None
    if all(v is not None for v in vparts):
        wi = (vparts[0] + vparts[1]) / cells
        limit = CUS * CLOCK_HZ / wi
        valu = {"wave_instr_per_cell_stage": wi, "issue_limited_value": limit, "frac": value / limit,
                "peak": "256 CUs x 2.4 GHz, one wave-instruction per CU per cycle"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
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
                   "cells": cells, "cfl": prob.cfl, "kappa": prob.kappa,
                   "boundary": "periodic" if prob.bc_x == 0 else "outflow"},
        "roofline": {"bound": "hbm", "kernel": "stage: k_points + k_cells + 1/3 of the step's dt reduction",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": stage_bytes,
                     "algorithmic_bytes_per_cell": BYTES_PER_CELL_STAGE, "avg_stage_us": stage_us,
                     "valu": valu, "per_kernel": per_kernel},
        "kernels_us": us,
        "stage_hbm_gbs": stage_bytes / t_stage / 1e9,
        "admissible": bool(st["admissible"]),
    }
    if not args.no_extra:
        import torch
        # the same steps replayed from a hipGraph (a one-instance batch)
        gstates = [af.to_device(u0)]
        gb = af.Batch([prob], gstates)
        for _ in range(args.warmup):
            gb.step()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(gb.stream)
        for _ in range(args.steps):
            gb.step()
        e1.record(gb.stream)
        torch.cuda.synchronize()
        out["graph_step_value"] = cells / (e0.elapsed_time(e1) * 1e-3 / stages)
        gb.close()
        del gstates

        # FP32-bulk stage on the same workload, and its difference from the
        # FP64 run after the same number of steps (L1 of rho and p, relative)
        ms32, st32, u32, us32 = stage_run(af, prob, u0, args, af.AF_FLAG_FP32_BULK)
        value32 = cells / (ms32 * 1e-3 / stages)

        def pressure(A):
            return (prob.gamma - 1) * (A[7] - 0.5 * (A[1] ** 2 + A[2] ** 2 + A[3] ** 2) / A[0]
                                       - 0.5 * (A[4] ** 2 + A[5] ** 2 + A[6] ** 2))

        l1_rho = float(abs(u32[0][0] - u64[0][0]).mean() / abs(u64[0][0]).mean())
        p64, p32 = pressure(u64[0]), pressure(u32[0])
        l1_p = float(abs(p32 - p64).mean() / abs(p64).mean())
        out["fp32_bulk"] = {"value": value32, "unit": UNIT, "speedup_vs_fp64": value32 / value,
                            "ms_per_step": ms32 / args.steps, "kernels_us": us32,
                            "admissible": bool(st32["admissible"]),
                            "min_rho": st32["min_rho"], "min_p": st32["min_p"],
                            "l1_rel_vs_fp64": {"rho": l1_rho, "p": l1_p},
                            "compared_after_steps": args.warmup + args.steps}

        # the Orszag-Tang vortex 512^2 (periodic; its states fit the 256 MB
        # Infinity Cache, so its rates are effective rates)
        if args.workload != "orszag_tang_512":
            ot = I.orszag_tang(512)
            ms_ot, st_ot, _, us_ot = stage_run(af, ot, I.sample(ot), args, 0)
            out["orszag_tang_512"] = {"value": ot.nx * ot.ny / (ms_ot * 1e-3 / stages), "unit": UNIT,
                                      "ms_per_step": ms_ot / args.steps, "kernels_us": us_ot,
                                      "admissible": bool(st_ot["admissible"])}

        copy = stream_copy_gbs(af)
        out["stream_copy"] = {"gbs": copy["gbs"], "buffer_bytes": copy["bytes"],
                              "stage_frac": achieved / copy["gbs"]}
    if not args.no_batch:
        out["batched"] = batched(af, I, args)
    if not args.no_adjoint:
        out["adjoint"] = adjoint(af, I, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, u0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
