"""af_mhd_step_noalloc (the step for callers that cannot allocate: scratch in
the library's static device array) against af_mhd_step of a context with a
caller-owned workspace, on two calls in a row, the second on a smaller
grid: every DoF and dt bitwise equal (the same kernels on the same inputs)."""
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


def reference_step(af, prob, u0, flags=0):
    import torch
    ctx = af.Context(prob, flags=flags)
    u = af.to_device(u0)
    ctx.af_mhd_step(u)
    torch.cuda.synchronize()
    out = af.to_host(u), float(ctx.dt_dev.item())
    ctx.close()
    return out


@pytest.mark.parametrize("flags", [0, 1], ids=["fp64", "fp32_bulk"])
def test_noalloc_step_equals_the_workspace_step(af, flags):
    import torch
    print(f"[noalloc] flags {flags}", flush=True)
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for prob in (I.random_shock(96, 80, seed=4, bc=I.OUTFLOW, field_jump=3.0), I.orszag_tang(40).with_size(40, 36)):
        u0 = I.sample(prob)
        want, want_dt = reference_step(af, prob, u0, flags)
        u = af.to_device(u0)
        af.af_mhd_step_noalloc(prob, u, dt_dev, flags=flags)
        torch.cuda.synchronize()
        assert float(dt_dev.item()) == want_dt
        for a, b in zip(af.to_host(u), want):
            assert np.array_equal(a, b), f"{prob.name} {prob.nx}x{prob.ny}"
        print(f"[noalloc] {prob.name} {prob.nx}x{prob.ny}: bitwise equal to af_mhd_step", flush=True)


def test_noalloc_step_rejects_what_does_not_fit(af):
    import torch
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    big = I.orszag_tang(512)
    u = af.empty_state(big)
    with pytest.raises(af.AfMhdError) as e:
        af.af_mhd_step_noalloc(big, u, dt_dev)
    assert e.value.code == af.AF_EINVAL and "48 MiB" in str(e.value)
    small = I.orszag_tang(16)
    with pytest.raises(af.AfMhdError) as e:
        af.af_mhd_step_noalloc(small, af.empty_state(small), dt_dev, flags=af.AF_FLAG_FUSED_DT)
    assert e.value.code == af.AF_EINVAL
