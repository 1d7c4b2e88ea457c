"""Batched ensembles through the C ABI: every instance of a batch (mixed
sizes, boundaries and gamma; flat, persistent or fused launches -- the
last one launch per stage whose cell tiles compute their own nine-point
sources; any cell-tile shape, plain launches or hipGraph replays) must be bitwise equal to the single-grid context's run
on that instance, step by step.

Each DoF's arithmetic is the same in both paths and the dt reduction is a
max (order-independent), so equality is exact.  The batch is also compared
with the CPU oracle directly, to the 1e-11 parity bar."""
import os
import sys
from dataclasses import replace

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def af():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    from paper_2506_04857_amd import af_mhd
    return af_mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_problems():
    return [
        I.random_smooth(20, 17, seed=3, bc=I.OUTFLOW),
        I.alfven(32),
        I.orszag_tang(40).with_size(40, 24),
        replace(I.random_shock(18, 15, seed=1, bc=I.PERIODIC, field_jump=3.0), kappa=0.0),
        I.blast_lowbeta(48),
        replace(I.random_smooth(13, 29, seed=4), bc_y=I.OUTFLOW),
    ]


def single_runs(af, probs, u0s, nsteps, flags):
    """States and dts of single-grid contexts after 1..nsteps steps."""
    import torch
    out = []
    for prob, u0 in zip(probs, u0s):
        ctx = af.Context(prob, flags=flags)
        u = af.to_device(u0)
        hist = []
        for _ in range(nsteps):
            ctx.af_mhd_step(u)
            torch.cuda.synchronize()
            hist.append((af.to_host(u), float(ctx.dt_dev.item())))
        ctx.close()
        out.append(hist)
    return out


def check_batch(af, probs, nsteps, flags=0, use_graph=True, tune_table=None, force_mode=None):
    """Bitwise equality with the single-grid runs, except in the fused mode,
    whose cell tiles form their nine-point sources with their own instruction
    selection (fused multiply-adds placed by the compiler in each context):
    there every field within 1e-14 of the single-grid run's scale (1e-6 for
    the FP32-bulk stage, whose sources are FP32 sums)."""
    import torch
    u0s = [I.sample(p) for p in probs]
    ref = single_runs(af, probs, u0s, nsteps, flags)
    states = [af.to_device(u) for u in u0s]
    b = af.Batch(probs, states, flags=flags, tune_table=tune_table)
    if force_mode is not None:
        b.set_launch_mode(force_mode)
    mode = b.launch_mode()  # with a tune table: the fastest of the three
    say(f"[batch] n={len(probs)} flags={flags} graph={use_graph} mode={b.launch_mode()} "
        f"tiles={[b.tile(m) for m in range(len(probs))]}")
    for n in range(nsteps):
        b.step(use_graph=use_graph)
        # eager work and a synchronisation between graph replays
        junk = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(junk) == 1000.0
        dts = b.dt_dev.cpu().numpy()
        for m in range(len(probs)):
            got = af.to_host(states[m])
            want, dt_want = ref[m][n]
            if mode == af.AF_BATCH_FUSED:
                tol = 1e-6 if flags & af.AF_FLAG_FP32_BULK else 1e-14
                assert abs(dts[m] - dt_want) <= 1e3 * tol * dt_want, f"step {n} instance {m}: dt {dts[m]!r}"
                for a, w in zip(got, want):
                    for c in range(8):
                        scale = max(float(np.max(np.abs(w[c]))), 1e-300)
                        err = float(np.max(np.abs(a[c] - w[c]))) / scale
                        assert err <= tol, f"step {n} instance {m} ({probs[m].name}) field {c}: {err:.3e}"
                continue
            assert dts[m] == dt_want, f"step {n} instance {m}: dt {dts[m]!r} vs {dt_want!r}"
            for a, w in zip(got, want):
                assert np.array_equal(a, w), f"step {n} instance {m} ({probs[m].name}) differs"
    cnt = b.counters()
    b.close()
    return cnt


def test_batch_graph_replays_equal_single_grid_runs(af):
    cnt = check_batch(af, mixed_problems(), 4, use_graph=True)
    assert cnt["n_not_admissible"] == 0


def test_batch_plain_launches_equal_single_grid_runs(af):
    check_batch(af, mixed_problems(), 2, use_graph=False)


def test_batch_fp32_equals_single_grid_fp32(af):
    check_batch(af, mixed_problems(), 3, flags=af.AF_FLAG_FP32_BULK, use_graph=True)


MODES = {"flat": 0, "persistent": 1, "fused": 2}


@pytest.mark.parametrize("mode", list(MODES))
def test_batch_launch_modes_equal_single_grid_runs(af, mode):
    # every launch mode, graph replays and plain launches, FP64 and FP32-bulk
    check_batch(af, mixed_problems(), 3, use_graph=True, force_mode=MODES[mode])
    check_batch(af, mixed_problems(), 1, use_graph=False, force_mode=MODES[mode])
    check_batch(af, mixed_problems(), 2, flags=af.AF_FLAG_FP32_BULK, use_graph=True, force_mode=MODES[mode])


def test_batch_mode_switch_recaptures_the_graph(af):
    # a graph captured in one mode is dropped when the mode changes
    import torch
    probs = mixed_problems()
    u0s = [I.sample(p) for p in probs]
    ref = single_runs(af, probs, u0s, 3, 0)
    states = [af.to_device(u) for u in u0s]
    b = af.Batch(probs, states)
    for n, mode in enumerate((MODES["persistent"], MODES["flat"], MODES["persistent"])):
        b.set_launch_mode(mode)
        assert b.launch_mode() == mode
        b.step(use_graph=True)
        torch.cuda.synchronize()
        for m in range(len(probs)):
            for a, w in zip(af.to_host(states[m]), ref[m][n][0]):
                assert np.array_equal(a, w), f"step {n} (mode {mode}) instance {m} differs"
    with pytest.raises(af.AfMhdError):
        b.set_launch_mode(7)
    b.close()


def test_batch_autotune_table(af, tmp_path):
    path = str(tmp_path / "tiles.txt")
    probs = mixed_problems()
    check_batch(af, probs, 2, use_graph=True, tune_table=path)
    with open(path) as fh:
        lines = [ln for ln in fh if ln.strip() and not ln.startswith("#")]
    classes = {(p.nx, p.ny, p.bc_x, p.bc_y) for p in probs}
    assert len(lines) == len(classes)
    say("[batch] tune table:\n" + "".join(lines))
    # a second batch reads the table and measures nothing new
    check_batch(af, probs, 1, use_graph=True, tune_table=path)
    with open(path) as fh:
        assert len([ln for ln in fh if ln.strip() and not ln.startswith("#")]) == len(classes)


def test_batch_of_the_orszag_tang_ensemble_recipe(af):
    # A few instances of the benchmark ensemble (sizes from {64..256}^2,
    # perturbed fields): batch vs single grid, bitwise, one graph step.
    probs = I.batched_orszag_tang(6)
    check_batch(af, probs, 1, use_graph=True)


def field_errors(got, want):
    out = []
    for g, w in zip(got, want):
        for c in range(8):
            scale = np.max(np.abs(w[c]))
            d = np.max(np.abs(g[c] - w[c]))
            out.append(d / scale if scale > 0 else d)
    return max(out)


@pytest.mark.parametrize("kind", ["mixed_kappa0_3_steps", "ensemble_kappa1_1_step"])
def test_batch_against_the_oracle(af, oracle, kind):
    # Every instance of a batch against the CPU oracle's steps directly (not
    # only through the single-grid context): the same dt and every field to
    # 1e-11 relative.  Multi-step comparisons use kappa = 0, where the scheme
    # is well conditioned; the shock sensor is compared over one step of the
    # benchmark ensemble's recipe.
    import torch
    if kind == "mixed_kappa0_3_steps":
        probs, nsteps = [replace(p, kappa=0.0) for p in mixed_problems()], 3
    else:
        probs, nsteps = I.batched_orszag_tang(4), 1
    u0s = [I.sample(p) for p in probs]
    states = [af.to_device(u) for u in u0s]
    b = af.Batch(probs, states)
    b.set_launch_mode(af.AF_BATCH_FUSED)
    refs = list(u0s)
    worst = 0.0
    for n in range(nsteps):
        b.step(use_graph=True)
        torch.cuda.synchronize()
        dts = b.dt_dev.cpu().numpy()
        for m, prob in enumerate(probs):
            refs[m], dt = oracle.step(prob, refs[m])
            assert abs(dts[m] - dt) <= 1e-12 * dt, f"step {n} instance {m}: dt {dts[m]!r} vs oracle {dt!r}"
            e = field_errors(af.to_host(states[m]), refs[m])
            worst = max(worst, e)
            assert e <= 1e-11, f"step {n} instance {m} ({prob.name} {prob.nx}x{prob.ny}): {e:.3e}"
    say(f"[batch] {kind}: {len(probs)} instances, {nsteps} steps, worst field rel err vs oracle {worst:.3e}")
    b.close()
