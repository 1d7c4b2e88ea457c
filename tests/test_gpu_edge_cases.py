"""Edge cases of the HIP stage through the C ABI: exact properties the
scheme has (constant states, mass conservation), degenerate physics
(B = 0), extreme aspect ratios, the smallest grids, a large grid, and
plane sets past 2^31 bytes (translation invariance of a tiled periodic
state), each against the FP64 oracle where one is computed."""
import sys
from dataclasses import replace

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I

pytestmark = pytest.mark.gpu

REL = 1e-11


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


def gpu_steps(af, prob, u0, nsteps, flags=0):
    import torch
    ctx = af.Context(prob, flags=flags)
    u = af.to_device(u0)
    masses = []
    for _ in range(nsteps):
        ctx.af_mhd_step(u)
        masses.append(ctx.af_mhd_stats(u)["mass"])
    torch.cuda.synchronize()
    st = ctx.af_mhd_stats(u)
    res = af.to_host(u)
    ctx.close()
    return res, st, np.array(masses)


@pytest.mark.parametrize("bc", [I.PERIODIC, I.OUTFLOW])
@pytest.mark.parametrize("flags", [0, 1], ids=["fp64", "fp32"])
def test_constant_state_preserved(af, bc, flags):
    # A constant state is a steady solution; the scheme keeps it to
    # rounding (the centre reconstruction and FVS differences cancel up to
    # a few ulp): 1e-13 relative after 100 steps in FP64, the FP32 level in
    # FP32-bulk.
    prob = I.constant_state(24, bc)
    u0 = I.sample(prob)
    got, st, _ = gpu_steps(af, prob, u0, 100, flags)
    e = max(np.max(np.abs(a - b)) / np.max(np.abs(b)) for a, b in zip(got, u0))
    say(f"[edge] constant state bc={bc} flags={flags}: drift {e:.2e}")
    assert e <= (1e-13 if flags == 0 else 2e-6)
    assert st["n_theta_active"] == 0 and st["n_point_limited"] == 0


def test_mass_conserved_with_active_limiters(af):
    # Periodic, flux limiter and scaling limiters active: the cell-average
    # update is in flux form with one flux per interface, so the total mass
    # stays constant to rounding.
    prob = replace(I.random_shock(40, 33, seed=1, bc=I.PERIODIC, field_jump=3.0), kappa=0.0)
    u0 = I.sample(prob)
    m0 = u0[0][0].sum() * prob.dx * prob.dy
    _, st, masses = gpu_steps(af, prob, u0, 20)
    drift = np.max(np.abs(masses - m0)) / abs(m0)
    say(f"[edge] mass drift over 20 limiter-active steps {drift:.2e}; theta-active {st['n_theta_active']}")
    assert st["n_theta_active"] > 0
    assert drift <= 1e-13


def test_hydrodynamic_limit_b_zero(af, oracle):
    # B = 0 everywhere: the Powell source and the magnetic terms vanish, the
    # fast speed is the sound speed; strong shock data.
    base = I.random_shock(22, 19, seed=4, bc=I.OUTFLOW)

    def prim(x, y, t):
        w = base.prim(x, y, t)
        w[4:7] = 0.0
        return w

    prob = replace(base, prim=prim)
    u0 = I.sample(prob)
    dt = oracle.dt(prob, u0)
    ref = oracle.stage(prob, 0, u0, u0, dt)
    import torch
    ctx = af.Context(prob)
    out = af.empty_state(prob)
    ctx.dt_dev.fill_(dt)
    ctx.af_mhd_stage(0, af.to_device(u0), af.to_device(u0), out)
    torch.cuda.synchronize()
    got = af.to_host(out)
    ctx.close()
    e = field_errors(got, ref).max()
    say(f"[edge] B = 0 shock: {e:.2e}")
    assert e <= REL
    assert all(np.all(g[4:7] == 0.0) for g in got)


@pytest.mark.parametrize("nx,ny,bc", [(4, 300, I.OUTFLOW), (300, 4, I.PERIODIC), (5, 4, I.PERIODIC),
                                      (4, 4, I.OUTFLOW), (33, 65, I.PERIODIC)])
def test_extreme_shapes_one_step(af, oracle, nx, ny, bc):
    prob = I.random_smooth(nx, ny, seed=nx * 1000 + ny, bc=bc)
    u0 = I.sample(prob)
    got, _, _ = gpu_steps(af, prob, u0, 1)
    ref, _ = oracle.step(prob, u0)
    e = field_errors(got, ref).max()
    say(f"[edge] {nx}x{ny} bc={bc}: {e:.2e}")
    assert e <= REL


def test_large_grid_one_step(af, oracle):
    # 2048 x 1536 Orszag-Tang (3.1M cells, several hundred tiles in each
    # direction): one SSP-RK3 step, every DoF against the oracle.
    prob = I.orszag_tang(2048).with_size(2048, 1536)
    u0 = I.sample(prob, gl=2)
    say("[edge] 2048x1536 one step (oracle takes a few seconds)")
    got, st, _ = gpu_steps(af, prob, u0, 1)
    ref, _ = oracle.step(prob, u0)
    e = field_errors(got, ref).max()
    say(f"[edge] 2048x1536: {e:.2e}")
    assert st["admissible"]
    assert e <= REL



def test_arrays_past_2gib_translation_invariance(af):
    # 16384 x 4096 cells: every [8][ny][nx] plane set is 4.3 GB, past 2^31
    # bytes, so any 32-bit byte offset would wrap.  The Orszag-Tang 512^2
    # data tiled 32 x 8 times is periodic with period 512 (and the domain
    # grows by powers of two, so dx and dy are the same numbers), hence one
    # stage of it must reproduce the 512^2 stage in every block, bit for bit.
    import torch
    small = I.orszag_tang(512)
    rx, ry = 32, 8
    big = replace(small, nx=512 * rx, ny=512 * ry, x1=small.x0 + rx * (small.x1 - small.x0),
                  y1=small.y0 + ry * (small.y1 - small.y0))
    assert big.dx == small.dx and big.dy == small.dy
    u0 = I.sample(small)
    dt = 1.0e-3
    ref = []
    ctx = af.Context(small)
    du = af.to_device(u0)
    out = af.empty_state(small)
    ctx.dt_dev.fill_(dt)
    ctx.af_mhd_stage(0, du, du, out)
    torch.cuda.synchronize()
    ref = af.to_host(out)
    ctx.close()
    del du, out
    say(f"[edge] {big.nx}x{big.ny}: {8 * big.nx * big.ny * 8 / 2**30:.1f} GiB per plane set")
    ctx = af.Context(big)
    dbig = tuple(torch.from_numpy(np.tile(a, (1, ry, rx))).to("cuda") for a in u0)
    out = af.empty_state(big)
    ctx.dt_dev.fill_(dt)
    ctx.af_mhd_stage(0, dbig, dbig, out)
    torch.cuda.synchronize()
    st = ctx.af_mhd_stats(out)
    del dbig
    worst = 0.0
    for q in range(4):
        got = out[q].cpu().numpy().reshape(8, ry, 512, rx, 512)
        worst = max(worst, float(np.max(np.abs(got - ref[q][:, None, :, None, :]))))
        del got
    ctx.close()
    say(f"[edge] tiled stage vs 512^2 stage: max |difference| {worst:.3e}")
    assert st["admissible"]
    assert worst == 0.0

def test_stream_copy_measurement_kernel(af):
    # the stream-copy kernel the bench compares bandwidth against
    import torch
    for n in (2, 1000, 3 * 2 ** 20 + 6):
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.zeros_like(src)
        af.stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
    with pytest.raises(af.AfMhdError):
        af.stream_copy(src[:-1], dst[:-1])  # odd length
