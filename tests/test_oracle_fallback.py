"""Pins of the round-off fallback (the closing remark of Section 4) and of
the centre limiter's value (Remark rmk:cell_center).

The fallback: when round-off leaves a limited state outside G although the
limiter aimed at rho >= eps_rho, p >= eps_p, the blending coefficient is
shrunk by 2^m 1e-8, m = 0, 1, ..., 9, until the state is in G.  Reading
(R19): each trial is taken from the original coefficient (not cumulative),
floored at 0; the first passing m wins; 0 (the safe state) if none passes;
the fallback acts only on leaving G itself (rho > 0, p > 0), not on missing
the eps bounds.  The cases are states whose scales differ a lot, as in the
paper's jets: |B|^2/2 up to ~1e9 against pressures down to 1e-8, so the
pressure of a blend is decided by the round-off of E - |m|^2/(2 rho) - |B|^2/2.

Each expected result is found here by brute force over the trial sequence,
with the state's membership in G evaluated in FP64 by the printed pressure
formula (the same operations as the oracle's, so the same decisions).  The
generators must produce cases with m = 0, with m >= 2 (which tells a
cumulative shrink apart), with the floor at 0 reached, and cases that miss
eps_p but stay in G (where the fallback must not act).
"""
import numpy as np
import pytest

from limiter_cases import (G, SOURCE_DT, box_cases, centre_cases, in_G, p_of, point_cases, source_cases)
from paper_2506_04857_amd.inputs import prim_to_cons

SHRINK = 1e-8


def first_passing(theta, make):
    """The fallback's result by brute force: (m, t) for the first trial
    t = max(theta - 2^m 1e-8, 0) with make(t) in G, (None, 0) if none."""
    for m in range(10):
        t = max(theta - 2.0 ** m * SHRINK, 0.0)
        if in_G(make(t)):
            return m, t
    return None, 0.0


class Tally:
    def __init__(self):
        self.m0 = self.m2 = self.floor = self.eps_only = self.fired = 0

    def add(self, m, t):
        self.fired += 1
        self.m0 += m == 0
        self.m2 += m is not None and m >= 2
        self.floor += t == 0.0

    def check(self):
        assert self.fired >= 20, vars(self)
        assert self.m0 > 0 and self.m2 > 0 and self.floor > 0, vars(self)
        assert self.eps_only > 0, vars(self)


def test_point_limiter_round_off_fallback(oracle):
    tally = Tally()
    for UH, UL in point_cases():
        out, nf = oracle.point_limiter(UH, UL, G)
        # Section 3.3 with "n" the LLF state: density step, then the blend
        rhoL, pL = UL[0], p_of(UL)
        er, ep = min(1e-13, rhoL), min(1e-13, pL)
        Us = UH.copy()
        if UH[0] < er:
            th1 = (rhoL - er) / (rhoL - UH[0])
            Us[0] = th1 * UH[0] + (1.0 - th1) * rhoL
        ps = p_of(Us)
        th2 = (pL - ep) / (pL - ps) if ps < ep else 1.0
        make = lambda t: t * Us + (1.0 - t) * UL  # noqa: E731
        if in_G(make(th2)):
            assert nf == 0 and np.array_equal(out, make(th2))
            tally.eps_only += p_of(make(th2)) < ep
            continue
        m, t = first_passing(th2, make)
        assert nf == 1
        np.testing.assert_array_equal(out, make(t))
        tally.add(m, t)
    tally.check()


def test_centre_limiter_round_off_fallback(oracle):
    tally = Tally()
    for Uc, A in centre_cases():
        out, nf = oracle.centre_limiter(Uc, A, G)
        # the remark's form theta~ Uc + (1 - theta~) A, two steps (R3)
        rhoA, pA = A[0], p_of(A)
        er, ep = min(1e-13, rhoA), min(1e-13, pA)
        th1 = (rhoA - er) / (rhoA - Uc[0]) if Uc[0] < er else 1.0
        Ur = th1 * Uc + (1.0 - th1) * A
        pr = p_of(Ur)
        th2 = (pA - ep) / (pA - pr) if pr < ep else 1.0
        make = lambda t: t * Ur + (1.0 - t) * A  # noqa: E731
        if in_G(make(th2)):
            assert nf == 0 and np.array_equal(out, make(th2))
            tally.eps_only += p_of(make(th2)) < ep
            continue
        m, t = first_passing(th2, make)
        assert nf == 1
        np.testing.assert_array_equal(out, make(t))
        tally.add(m, t)
    tally.check()


def test_source_limiter_round_off_fallback(oracle):
    # Step (1) of the flux limiter with no flux correction (F^s = F^LLF):
    # A^{Lim,1} = theta A^src + (1 - theta) A^LLF with the fallback on theta.
    tally = Tally()
    dt, dx, dy = SOURCE_DT, 0.5, 0.25
    Fl = np.zeros((4, 8))
    for A, S_s, S_llf in source_cases():
        th, lam, A1, nf = oracle.cell_limiter(A, Fl, Fl, S_s, S_llf, dt, dx, dy, G)
        Allf, Asrc = A - dt * S_llf, A - dt * S_s
        pL = p_of(Allf)
        ep = min(1e-13, pL)
        ps = p_of(Asrc)
        th0 = (pL - ep) / (pL - ps) if ps < ep else 1.0
        make = lambda t: t * Asrc + (1.0 - t) * Allf  # noqa: E731
        if in_G(make(th0)):
            assert nf == 0 and th == th0
            tally.eps_only += p_of(make(th0)) < ep
            continue
        m, t = first_passing(th0, make)
        assert nf >= 1 and th == t, (th, t, m)
        np.testing.assert_array_equal(A1, make(t))
        tally.add(m, t)
    tally.check()


def box_ok(A1, H, L):
    """All 15 non-trivial corners A1 + sum_{I in K} L_I H_I of the box in G
    (terms summed in the order L, R, D, U)."""
    for k in range(1, 16):
        D = np.zeros(8)
        for I in range(4):
            if k >> I & 1:
                D = D + L[I] * H[I]
        if not in_G(A1 + D):
            return False
    return True


def test_flux_limiter_box_round_off_fallback(oracle):
    fired = m0 = m2 = floor = 0
    for A1, H, er, ep in box_cases():
        lam, info = oracle.flux_limiter_box(A1, H, G, er, ep)
        pre = info["lambda_before_fallback"]
        # the box before the fallback: the printed density box times the
        # smallest vertex root (where no root was needed, the density box)
        neg = sum(h for h in H[:, 0] if h < 0)
        Lr = np.array([min(1.0, (A1[0] - er) / (1e-12 - neg)) if H[I, 0] < 0 else 1.0 for I in range(4)])
        assert np.all(pre <= Lr)
        if info["n_newton"] == 0:
            np.testing.assert_array_equal(pre, Lr)
            assert info["n_fallback"] == 0
            continue
        if box_ok(A1, H, pre):
            assert info["n_fallback"] == 0
            np.testing.assert_array_equal(lam, pre)
            continue
        assert info["n_fallback"] == 1
        m = None
        for mm in range(10):
            L = np.maximum(pre - 2.0 ** mm * SHRINK, 0.0)
            if box_ok(A1, H, L):
                m = mm
                break
        want = L if m is not None else np.zeros(4)
        np.testing.assert_array_equal(lam, want)
        fired += 1
        m0 += m == 0
        m2 += m is not None and m >= 2
        floor += bool(np.any(want == 0.0))
    assert fired >= 20 and m0 > 0 and m2 > 0 and floor > 0, (fired, m0, m2, floor)


# ------------------------------------------------- the centre limiter's value
def bisect_largest(f, lo=0.0, hi=1.0):
    """Largest t in [0, 1] with f(t) >= 0 for f(0) >= 0, by bisection."""
    if f(hi) >= 0:
        return hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) >= 0 else (lo, mid)
    return lo


def on_segment(C, A, Uc):
    """The coefficient t with C = t Uc + (1 - t) A, asserting that all eight
    components (density included) share it: the remark's printed form."""
    d = Uc - A
    t = (C - A) @ d / (d @ d)
    np.testing.assert_allclose(C, A + t * d, rtol=1e-12, atol=1e-12 * np.abs(A).max())
    return t


def test_centre_limiter_density_active_value(oracle):
    # Uc with negative density, zero momentum and a large energy: only the
    # density bound binds, rho is linear along [A, Uc], and the largest
    # feasible coefficient is (rho(A) - eps) / (rho(A) - rho(Uc)).
    rng = np.random.default_rng(2506 + 75)
    for _ in range(200):
        A = prim_to_cons(np.array([rng.uniform(0.5, 2), 0, 0, 0, *rng.uniform(-1, 1, 3), rng.uniform(0.5, 2)]), G)
        Uc = A.copy()
        Uc[0] = -rng.uniform(0.01, 2.0)
        Uc[4:7] = A[4:7]
        Uc[7] = A[7] * rng.uniform(1.0, 3.0)
        C, nf = oracle.centre_limiter(Uc, A, G)
        assert nf == 0
        t = on_segment(C, A, Uc)
        er, ep = min(1e-13, A[0]), min(1e-13, p_of(A))
        t_max = bisect_largest(lambda s: min(((1 - s) * A[0] + s * Uc[0]) - er,
                                             p_of((1 - s) * A + s * Uc) - ep if (1 - s) * A[0] + s * Uc[0] > 0
                                             else -1.0))
        assert t == pytest.approx(t_max, abs=1e-12)
        assert C[0] == pytest.approx(er, abs=1e-15)


def test_centre_limiter_pressure_active_value(oracle):
    # Uc with the cell average's momentum and field but a lower energy: the
    # pressure is linear along [A, Uc], so the scaling fraction is the
    # largest feasible coefficient.
    rng = np.random.default_rng(2506 + 76)
    for _ in range(200):
        A = prim_to_cons(np.array([rng.uniform(0.5, 2), *rng.uniform(-1, 1, 6), rng.uniform(0.01, 2)]), G)
        Uc = A.copy()
        Uc[0] = A[0] * rng.uniform(0.5, 1.5)
        Uc[1:4] = A[1:4] * Uc[0] / A[0]  # same velocity: |m|^2/(2 rho) linear in the blend
        Uc[7] = A[7] - 0.5 * (A[1:4] @ A[1:4]) / A[0] + 0.5 * (Uc[1:4] @ Uc[1:4]) / Uc[0] \
            - rng.uniform(1.5, 10.0) * p_of(A) / (G - 1)
        assert p_of(Uc) < 0
        C, nf = oracle.centre_limiter(Uc, A, G)
        assert nf == 0
        t = on_segment(C, A, Uc)
        ep = min(1e-13, p_of(A))
        t_max = bisect_largest(lambda s: p_of((1 - s) * A + s * Uc) - ep)
        assert t == pytest.approx(t_max, abs=1e-12)


def test_centre_limiter_general_value(oracle):
    # Both bounds violated, general states: the result keeps the printed
    # one-coefficient form, is feasible, and is no further from Uc than the
    # largest feasible coefficient.
    rng = np.random.default_rng(2506 + 77)
    n_active = 0
    for _ in range(400):
        A = prim_to_cons(np.array([rng.uniform(0.2, 2), *rng.uniform(-1, 1, 6), rng.uniform(1e-3, 1)]), G)
        Uc = A + rng.normal(size=8) * np.abs(A) * 10 ** rng.uniform(-1, 0.7)
        C, nf = oracle.centre_limiter(Uc, A, G)
        assert nf == 0
        er, ep = min(1e-13, A[0]), min(1e-13, p_of(A))
        if Uc[0] >= er and p_of(Uc) >= ep:
            assert np.array_equal(C, Uc)
            continue
        n_active += 1
        t = on_segment(C, A, Uc)
        assert 0.0 <= t <= 1.0 + 1e-12
        assert C[0] >= er * (1 - 1e-12) and p_of(C) >= ep - 1e-14 * np.abs(C).max() ** 2
        rho = lambda s: (1 - s) * A[0] + s * Uc[0]  # noqa: E731
        t_max = bisect_largest(lambda s: min(rho(s) - er, p_of((1 - s) * A + s * Uc) - ep) if rho(s) > 0 else -1.0)
        assert t <= t_max + 1e-12
    assert n_active > 100
