"""FP32-bulk stage (AF_FLAG_FP32_BULK) through the C ABI against the FP64
oracle.

The bulk arithmetic (fluxes, wave speeds, FVS and LLF sums, sensor, source
sums) runs in FP32 with unit roundoff u = 2^-24 = 6e-8; storage, pressure
recovery, the centre value, the U + dt RHS accumulation and the limiters
stay FP64.  One stage adds dt times an FP32 right-hand side whose rounding
error is a few u times the largest flux magnitude over h; with
dt (|v| + c_f) / h <= CFL = 0.2 that is a few u (~1e-7) of the state scale
per stage, so single stages are held to 2e-6 of each field's scale on data
whose fields have comparable scales.  The limiters take their decisions in
FP64 from FP32 inputs, so on shock data where they act (scaling limiters,
the flux limiter's box and Newton roots) single stages are held to the same
bar; over many steps limiter-active data are checked for positivity and
for L1 errors of rho and p.
"""
import sys
from dataclasses import replace

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_STAGE = 2e-6


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


def field_errors(gpu, ref):
    out = []
    for g, r in zip(gpu, ref):
        for c in range(8):
            scale = np.max(np.abs(r[c]))
            d = np.max(np.abs(g[c] - r[c]))
            out.append(d / scale if scale > 0 else d)
    return np.array(out)


def fp32_stage(af, prob, k, un, uk, dt):
    import torch
    ctx = af.Context(prob, flags=af.AF_FLAG_FP32_BULK)
    dun, duk = af.to_device(un), af.to_device(uk)
    out = af.empty_state(prob)
    ctx.dt_dev.fill_(dt)
    ctx.af_mhd_stage(k, dun, duk, out)
    torch.cuda.synchronize()
    res = af.to_host(out)
    st = ctx.af_mhd_stats(out)
    ctx.close()
    return res, st


def fp32_run(af, prob, u0, nsteps, dts=None):
    """nsteps SSP-RK3 steps; with dts given, those time steps (so that the
    comparison isolates the stage arithmetic)."""
    import torch
    ctx = af.Context(prob, flags=af.AF_FLAG_FP32_BULK)
    u = af.to_device(u0)
    s1, s2 = af.empty_state(prob), af.empty_state(prob)
    for n in range(nsteps):
        if dts is None:
            ctx.af_mhd_step(u)
        else:
            ctx.dt_dev.fill_(dts[n])
            ctx.af_mhd_stage(0, u, u, s1)
            ctx.af_mhd_stage(1, u, s1, s2)
            ctx.af_mhd_stage(2, u, s2, u)
    torch.cuda.synchronize()
    st = ctx.af_mhd_stats(u)
    res = af.to_host(u)
    ctx.close()
    return res, st


def pressure(A, gamma):
    rho = A[0]
    return (gamma - 1) * (A[7] - 0.5 * (A[1] ** 2 + A[2] ** 2 + A[3] ** 2) / rho - 0.5 * (A[4] ** 2 + A[5] ** 2 + A[6] ** 2))


SINGLE = [
    ("smooth_13x9_periodic", lambda: I.random_smooth(13, 9, seed=1)),
    ("smooth_12x10_outflow", lambda: I.random_smooth(12, 10, seed=2, bc=I.OUTFLOW)),
    ("orszag_tang_70x37", lambda: I.orszag_tang(70).with_size(70, 37)),
    ("alfven_32", lambda: I.alfven(32)),
]


@pytest.mark.parametrize("name,make", SINGLE, ids=[s[0] for s in SINGLE])
def test_fp32_single_stages(af, oracle, name, make):
    prob = make()
    un = I.sample(prob)
    dt = oracle.dt(prob, un)
    uk = oracle.stage(prob, 0, un, un, dt)
    for k in (0, 1, 2):
        src = un if k == 0 else uk
        ref = oracle.stage(prob, k, un, src, dt)
        got, st = fp32_stage(af, prob, k, un, src, dt)
        e = field_errors(got, ref).max()
        say(f"[fp32] {name} stage {k}: worst field rel err {e:.2e}")
        assert st["admissible"]
        assert e <= TOL_STAGE, f"{name} k={k}: {e:.3e}"


# (name, problem, whether the flux limiter's coefficients and Newton roots act)
SHOCKS = [
    ("shock_24x21_outflow", lambda: I.random_shock(24, 21, seed=1, bc=I.OUTFLOW), True),
    ("shock_24x22_periodic", lambda: I.random_shock(24, 22, seed=5, bc=I.PERIODIC), True),
    ("blast_lowbeta_48", lambda: I.blast_lowbeta(48), False),
]


@pytest.mark.parametrize("name,make,flux_limiter", SHOCKS, ids=[s[0] for s in SHOCKS])
def test_fp32_single_stages_with_active_limiters(af, oracle, name, make, flux_limiter):
    # Shock data on which the point and centre scaling limiters act, and in
    # two cases the flux limiter's coefficients and Newton roots (the
    # oracle's counters say so): each FP32-bulk stage against the FP64
    # oracle's, to the same bar as on smooth data (measured: below 5e-7).
    prob = make()
    un = I.sample(prob)
    dt = oracle.dt(prob, un)
    cnt = oracle.Counters()
    uk = oracle.stage(prob, 0, un, un, dt)
    for k in (0, 1, 2):
        src = un if k == 0 else uk
        ref = oracle.stage(prob, k, un, src, dt, counters=cnt)
        got, st = fp32_stage(af, prob, k, un, src, dt)
        e = field_errors(got, ref).max()
        say(f"[fp32] {name} stage {k}: worst field rel err {e:.2e}")
        assert st["admissible"]
        assert e <= TOL_STAGE, f"{name} k={k}: {e:.3e}"
    say(f"[fp32] {name}: oracle limited points {cnt.n_point_limited}, centres {cnt.n_centre_limited}, "
        f"theta active {cnt.n_theta_active}, Newton {cnt.n_newton}")
    assert cnt.n_point_limited > 0 and cnt.n_centre_limited > 0
    if flux_limiter:
        assert cnt.n_theta_active > 0 and cnt.n_newton > 0


def test_fp32_alfven_100_steps_keeps_the_accuracy(af, oracle):
    # Same dt sequence as the oracle; the FP32 rounding adds ~1e-7 per
    # stage, far below the scheme's own error on 32^2 (~1e-4 in L1), so the
    # L1 error against the exact solution (the initial data translated by
    # the wave, here a whole number of periods is not reached: compare with
    # the FP64 oracle's own L1 error at the same time) is unchanged.
    prob = I.alfven(32)
    u0 = I.sample(prob)
    ref, dts = u0, []
    for _ in range(100):
        ref, d = oracle.step(prob, ref)
        dts.append(d)
    got, st = fp32_run(af, prob, u0, 100, dts)
    e = field_errors(got, ref).max()
    exact = I.sample(prob, t=float(np.sum(dts)))
    l1_32 = np.abs(got[0] - exact[0]).mean(axis=(1, 2))
    l1_64 = np.abs(ref[0] - exact[0]).mean(axis=(1, 2))
    say(f"[fp32] alfven 32 x 100 steps: vs oracle {e:.2e}; L1 vs exact fp32 {l1_32.max():.3e} fp64 {l1_64.max():.3e}")
    assert st["admissible"]
    assert e <= 1e-5
    assert np.all(np.abs(l1_32 - l1_64) <= 1e-3 * l1_64.max() + 1e-9)


def test_fp32_blast_positivity_and_l1(af, oracle):
    # Low-beta blast (ambient beta 2.5e-4) at 128^2: the point and centre
    # scaling limiters act at the blast front every step.  FP32-bulk keeps rho and p positive and
    # its L1 errors against the FP64 oracle stay at the FP32 level.
    prob = I.blast_lowbeta(128)
    u0 = I.sample(prob)
    ref, dts = u0, []
    c = oracle.Counters()
    for _ in range(20):
        ref, d = oracle.step(prob, ref, counters=c)
        dts.append(d)
    got, st = fp32_run(af, prob, u0, 20, dts)
    rho32, rho64 = got[0][0], ref[0][0]
    p32, p64 = pressure(got[0], prob.gamma), pressure(ref[0], prob.gamma)
    l1_rho = np.abs(rho32 - rho64).mean() / np.abs(rho64).mean()
    l1_p = np.abs(p32 - p64).mean() / np.abs(p64).mean()
    say(f"[fp32] blast 128 x 20 steps: min rho {st['min_rho']:.4e} (fp64 {min(a[0].min() for a in ref):.4e}), "
        f"min p {st['min_p']:.4e}, L1 rel rho {l1_rho:.2e}, L1 rel p {l1_p:.2e}, "
        f"points limited {st['n_point_limited']} (fp64 {c.n_point_limited}), "
        f"centres limited {st['n_centre_limited']} (fp64 {c.n_centre_limited})")
    assert c.n_point_limited > 0 and c.n_centre_limited > 0  # the limiters act in this run
    assert st["n_point_limited"] > 0 and st["n_centre_limited"] > 0
    assert st["admissible"] and st["n_not_admissible"] == 0
    assert st["min_rho"] > 0 and st["min_p"] > 0
    assert l1_rho <= 1e-5 and l1_p <= 1e-4


@pytest.mark.timeout(600)
def test_fp32_blast_1024_against_the_fp64_oracle(af, oracle):
    # The low-beta blast at its full size (1024^2, outflow, kappa = 1), 10
    # steps with the oracle's dt sequence: min rho, min p and the L1 errors
    # of rho and p of the FP32-bulk run against the FP64 oracle.
    prob = I.blast_lowbeta(1024)
    u0 = I.sample(prob)
    ref, dts = u0, []
    c = oracle.Counters()
    say("[fp32] blast 1024: oracle 10 steps")
    for _ in range(10):
        ref, d = oracle.step(prob, ref, counters=c)
        dts.append(d)
    say("[fp32] blast 1024: fp32-bulk 10 steps")
    got, st = fp32_run(af, prob, u0, 10, dts)
    rho32, rho64 = got[0][0], ref[0][0]
    p32, p64 = pressure(got[0], prob.gamma), pressure(ref[0], prob.gamma)
    l1_rho = np.abs(rho32 - rho64).mean() / np.abs(rho64).mean()
    l1_p = np.abs(p32 - p64).mean() / np.abs(p64).mean()
    min_rho64 = min(a[0].min() for a in ref)
    min_p64 = min(pressure(a, prob.gamma).min() for a in ref)
    say(f"[fp32] blast 1024 x 10 steps: min rho {st['min_rho']:.6e} (fp64 oracle {min_rho64:.6e}), "
        f"min p {st['min_p']:.6e} (fp64 oracle {min_p64:.6e}), L1 rel rho {l1_rho:.2e}, L1 rel p {l1_p:.2e}, "
        f"points limited {st['n_point_limited']} (fp64 {c.n_point_limited}), "
        f"centres limited {st['n_centre_limited']} (fp64 {c.n_centre_limited})")
    assert st["admissible"] and st["n_not_admissible"] == 0
    assert st["min_rho"] > 0 and st["min_p"] > 0
    assert st["min_rho"] == pytest.approx(min_rho64, rel=1e-4)
    assert l1_rho <= 1e-5 and l1_p <= 1e-4


def test_fp32_differs_from_fp64_only_by_rounding(af):
    # The two precisions run the same scheme: on OT 128^2 after 10 steps
    # their difference is at the FP32 rounding level, far above FP64's.
    import torch
    prob = replace(I.orszag_tang(128), kappa=0.0)
    u0 = I.sample(prob)
    res = {}
    for name, flags in (("fp64", 0), ("fp32", af.AF_FLAG_FP32_BULK)):
        ctx = af.Context(prob, flags=flags)
        u = af.to_device(u0)
        ctx.dt_dev.fill_(1e-3)
        s1, s2 = af.empty_state(prob), af.empty_state(prob)
        for _ in range(10):
            ctx.af_mhd_stage(0, u, u, s1)
            ctx.af_mhd_stage(1, u, s1, s2)
            ctx.af_mhd_stage(2, u, s2, u)
        torch.cuda.synchronize()
        res[name] = af.to_host(u)
        ctx.close()
    e = field_errors(res["fp32"], res["fp64"]).max()
    say(f"[fp32] OT 128 kappa=0 10 steps: fp32 vs fp64 {e:.2e}")
    assert 1e-12 < e <= 1e-5
