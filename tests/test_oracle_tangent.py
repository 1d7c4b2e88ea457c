"""Pins of the tangent oracle (the oracle's source built on forward-mode dual
numbers, the reference of the adjoint): its values are the plain oracle's,
bit for bit, and its derivatives are the central finite differences of the
plain oracle wherever the stage is differentiable (smooth data, sensor on and
off, periodic and outflow, one stage and several steps).  Where the sensor
sits on a kink (div v or div Bbar zero up to rounding, as on the Alfven
wave of the adjoint workload) finite differences average over the kink and the dual numbers take the
branch of the value; that case is shown, not hidden."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I


def rnd(rng, u):
    return tuple(rng.standard_normal(a.shape) for a in u)


def axpy(a, x, y):
    return tuple(xx * a + yy for xx, yy in zip(x, y))


def rel_err(fd, t):
    return max(np.max(np.abs(f - x)) for f, x in zip(fd, t)) / max(np.max(np.abs(x)) for x in t)


CASES = [
    ("smooth_periodic_k0", lambda: replace(I.random_smooth(12, 10, seed=3), kappa=0.0)),
    ("smooth_periodic_k1", lambda: I.random_smooth(12, 10, seed=3)),
    ("smooth_outflow_k0", lambda: replace(I.random_smooth(11, 9, seed=5, bc=I.OUTFLOW), kappa=0.0)),
    ("smooth_outflow_k1", lambda: I.random_smooth(11, 9, seed=5, bc=I.OUTFLOW)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_tangent_stage_values_and_central_differences(oracle, name, make):
    prob = make()
    rng = np.random.default_rng(7)
    u0 = I.sample(prob)
    dt = oracle.dt(prob, u0)
    for k in range(3):
        uk = oracle.stage(prob, 0, u0, u0, dt) if k else u0
        dn = [rnd(rng, u0) for _ in range(2)]
        dk = [rnd(rng, u0) for _ in range(2)] if k else dn
        out, douts = oracle.tangent_stage(prob, k, u0, dn, uk, dk, dt)
        ref = oracle.stage(prob, k, u0, uk, dt)
        assert all(np.array_equal(a, b) for a, b in zip(out, ref)), "tangent values differ from the oracle"
        h = 1e-6
        for d in range(2):
            p = oracle.stage(prob, k, axpy(h, dn[d], u0), axpy(h, dk[d], uk), dt)
            m = oracle.stage(prob, k, axpy(-h, dn[d], u0), axpy(-h, dk[d], uk), dt)
            fd = [(a - b) / (2 * h) for a, b in zip(p, m)]
            assert rel_err(fd, douts[d]) <= 1e-7, (k, d, rel_err(fd, douts[d]))


def test_tangent_run_matches_central_differences(oracle):
    # Several steps of the adjoint workload's wave (16^2, sensor off) with
    # a fixed dt sequence: d J / d u0 along unit-Gaussian directions.
    prob = replace(I.alfven_perturbed(16), kappa=0.0)
    u0 = I.sample(prob)
    dts, u = [], u0
    for _ in range(5):
        u, d = oracle.step(prob, u)
        dts.append(d)

    def J(s):
        return 0.5 * np.sum((s[0][0] - 1.0) ** 2)

    def run(s):
        for d in dts:
            s, _ = oracle.step(prob, s, fixed_dt=d)
        return s

    dirs = I.adjoint_directions(prob, 3)
    uT, du = oracle.tangent_run(prob, u0, dirs, dts)
    assert all(np.array_equal(a, b) for a, b in zip(uT, run(u0)))
    h = 1e-7
    for v, dv in zip(dirs, du):
        g_t = np.sum((uT[0][0] - 1.0) * dv[0][0])
        g_fd = (J(run(axpy(h, v, u0))) - J(run(axpy(-h, v, u0)))) / (2 * h)
        assert abs(g_t - g_fd) <= 1e-7 * abs(g_t), (g_t, g_fd)


def test_tangent_at_sensor_kinks_is_one_sided(oracle):
    # The adjoint workload's wave: div v and the numerator of phi3 (the
    # central divergence of Bbar) are zero up to rounding, so the sensor sits
    # on the kinks of max(., 0) and |.|.  The tangent takes the branch the
    # value takes; central differences straddle the kinks and average the
    # slopes.  With the sensor off both agree.
    prob = I.alfven_perturbed(16)
    u0 = I.sample(prob)
    dt = oracle.dt(prob, u0)
    rng = np.random.default_rng(3)
    v = rnd(rng, u0)
    h = 1e-6
    errs = {}
    for kappa in (0.0, 1.0):
        p_ = replace(prob, kappa=kappa)
        _, d = oracle.tangent_stage(p_, 0, u0, [v], u0, [v], dt)
        p = oracle.stage(p_, 0, axpy(h, v, u0), axpy(h, v, u0), dt)
        m = oracle.stage(p_, 0, axpy(-h, v, u0), axpy(-h, v, u0), dt)
        errs[kappa] = rel_err([(a - b) / (2 * h) for a, b in zip(p, m)], d[0])
    assert errs[0.0] <= 1e-8
    assert errs[1.0] > 1e-2
