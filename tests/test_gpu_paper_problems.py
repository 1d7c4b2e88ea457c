"""The paper's two-dimensional tests on the GPU through the C ABI: accuracy
ladders (third order on the sine wave and the CP Alfven wave; the near-vacuum
vortex with minimum pressure 5.3e-12 stays positive and converges at
almost third order), the paper's own Orszag-Tang vortex at 400^2 to t = 2
with the two div B diagnostics recorded over time (Section 4: they level
off), and the paper's blast at 400^2 (positivity).  L1 errors are means over cells of |cell average -
exact cell average| (5x5 Gauss-Legendre)."""
import sys

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


def p_of(A, g):
    return (g - 1) * (A[7] - 0.5 * (A[1] ** 2 + A[2] ** 2 + A[3] ** 2) / A[0] - 0.5 * (A[4] ** 2 + A[5] ** 2 + A[6] ** 2))


def ladder(af, make, ns, T, comps):
    import torch
    errs = []
    for n in ns:
        prob = make(n)
        s = af.Solver(prob)
        u = af.to_device(I.sample(prob))
        t, steps = s.run(u, T)
        st = s.af_mhd_stats(u)
        s.close()
        torch.cuda.synchronize()
        got = af.to_host(u)
        ex = I.sample(prob, t)
        e = np.mean(np.abs(got[0] - ex[0]), axis=(1, 2))[comps]
        errs.append(e)
        say(f"[paper] {prob.name} n={n} steps={steps} t={t:.4f} L1={e} admissible={st['admissible']} "
            f"min_p={st['min_p']:.3e}")
        assert st["admissible"]
    errs = np.array(errs)
    return errs, np.log2(errs[:-1] / errs[1:])


def test_sine_wave_third_order(af):
    errs, rates = ladder(af, I.sine_wave, (32, 64, 128, 256), 0.1, [0, 7])
    say(f"[paper] sine wave rates {rates.tolist()}")
    assert np.all(rates[-1] > 2.8), rates


def test_alfven_wave_third_order_over_a_period(af):
    # the exact solution at t = 1 equals the initial data
    errs, rates = ladder(af, I.alfven, (32, 64, 128), 1.0, [1, 2, 3, 4, 5, 6])
    say(f"[paper] Alfven rates {rates.tolist()}")
    assert np.all(rates[-1] > 2.75), rates


def test_vortex_stays_positive_and_converges(af):
    # The paper's accuracy test: minimum pressure 5.3e-12 at the centre
    # (reading R21), T = 0.1, the PP limiters active.  Read without the shock
    # sensor (R29): with kappa = 1, phi3's denominator |B1 + B2| vanishes on
    # the vortex's diagonal and the sensor blends towards first order there
    # (measured: rates ~1).
    from dataclasses import replace
    errs, rates = ladder(af, lambda n: replace(I.vortex(n), kappa=0.0), (64, 128, 256, 512), 0.1, [0, 7])
    say(f"[paper] vortex rates {rates.tolist()}")
    assert np.all(rates[-1] > 2.4), rates
    # positivity with the sensor on as well
    _, _ = ladder(af, I.vortex, (256,), 0.1, [0, 7])


def test_paper_orszag_tang_400_divb_history(af):
    # Section 4: both discrete divergences grow while the vortex steepens and
    # then level off ("almost a plateau").  Measured: div1 0.29 (t = 0.25),
    # 0.78 (t = 1), 0.84 (t = 2).
    import torch
    from dataclasses import replace
    prob = replace(I.orszag_tang_paper(400), t_final=2.0)
    s = af.Solver(prob)
    u = af.to_device(I.sample(prob))
    hist, t = [], 0.0
    for k in range(8):
        t, _ = s.run(u, 0.25 * (k + 1), t0=t)
        d = s.af_mhd_divb(u).cpu().numpy()
        st = s.af_mhd_stats(u)
        hist.append((t, float(d[0]), float(d[1]), st["min_p"]))
        assert st["admissible"]
    s.close()
    torch.cuda.synchronize()
    for row in hist:
        say("[paper] OT400 t=%.3f div1=%.4e div2=%.4e min_p=%.3e" % row)
    for q in (1, 2):
        d = np.array([h[q] for h in hist])
        # growth over t in [1, 2] is a small part of the growth over [0.25, 1]
        assert d[7] - d[3] < 0.2 * (d[3] - d[0]), d


def test_paper_blast_400_positive(af):
    import torch
    prob = I.blast_paper(400)
    s = af.Solver(prob)
    u = af.to_device(I.sample(prob))
    t, steps = s.run(u, prob.t_final)
    st = s.af_mhd_stats(u)
    s.close()
    torch.cuda.synchronize()
    say(f"[paper] blast 400^2 t={t:.4f} steps={steps} min_rho={st['min_rho']:.3e} min_p={st['min_p']:.3e} "
        f"limited points {st['n_point_limited']} theta-active {st['n_theta_active']}")
    assert st["admissible"] and st["min_p"] > 0 and st["min_rho"] > 0
    assert abs(t - prob.t_final) < 1e-12
