"""Pins of the positivity limiters (Sections 3.2 and 3.3): brute force over
the admissible box, an independent root of the pressure cubic, and the
scaling limiter's guarantees."""
import numpy as np
import pytest

from paper_2506_04857_amd.inputs import prim_to_cons

G = 1.4


def p_of(U, g=G):
    return (g - 1) * (U[..., 7] - (U[..., 1] ** 2 + U[..., 2] ** 2 + U[..., 3] ** 2) / (2 * U[..., 0])
                      - (U[..., 4] ** 2 + U[..., 5] ** 2 + U[..., 6] ** 2) / 2)


def cases(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        w = np.array([rng.uniform(0.2, 2), *rng.uniform(-1, 1, 3), *rng.uniform(-1, 1, 3), rng.uniform(1e-3, 0.5)])
        A1 = prim_to_cons(w, G)
        scale = 10 ** rng.uniform(-2, 0.5)
        H = rng.normal(size=(4, 8)) * scale * np.abs(A1)[None, :] + rng.normal(size=(4, 8)) * 0.05 * scale
        out.append((A1, H))
    return out


def eps_of(A1):
    return min(1e-13, A1[0]), min(1e-13, p_of(A1))


def test_flux_limiter_box_is_admissible_by_brute_force(oracle):
    n_root = n_fb = 0
    for A1, H in cases(21, 250):
        er, ep = eps_of(A1)
        lam, info = oracle.flux_limiter_box(A1, H, G, er, ep)
        n_root += info["n_newton"]
        n_fb += info["n_fallback"]
        assert np.all(lam >= 0) and np.all(lam <= 1)
        grid = np.linspace(0, 1, 5)
        T = np.stack(np.meshgrid(grid, grid, grid, grid, indexing="ij"), -1).reshape(-1, 4) * lam[None, :]
        W = A1[None, :] + T @ H
        assert np.all(W[:, 0] >= er * (1 - 1e-12))
        # p >= eps_p up to the round-off of forming and evaluating these states
        # (terms of size |A1| + sum |H_I| cancel in them)
        tol = 1e-14 * (np.max(np.abs(A1)) + np.abs(H).sum(0).max()) ** 2
        assert np.all(p_of(W) >= ep - tol), (lam, p_of(W).min())
        assert np.all(p_of(W) > 0)
        # the box is the largest of its kind: some corner touches a bound
        # unless the whole unit box is admissible
        if np.any(lam < 1):
            corners = A1[None, :] + (np.stack(np.meshgrid(*[[0, 1]] * 4, indexing="ij"), -1).reshape(-1, 4)
                                     * lam[None, :]) @ H
            slack = np.minimum((corners[:, 0] - er) / max(A1[0], 1e-300), (p_of(corners) - ep) / max(p_of(A1), 1e-300))
            assert slack.min() < 1e-6
    assert n_root > 20  # the pressure shrink is exercised
    assert n_fb == 0  # the round-off fallback must not be what makes the box admissible


def test_flux_limiter_box_is_one_when_nothing_is_violated(oracle):
    A1 = prim_to_cons(np.array([1.0, 0.1, 0.2, 0.0, 0.3, 0.1, 0.0, 1.0]), G)
    H = 1e-3 * np.abs(np.random.default_rng(3).normal(size=(4, 8)))  # density increases, tiny changes
    lam, info = oracle.flux_limiter_box(A1, H, G, *eps_of(A1))
    assert np.all(lam == 1.0) and info["n_newton"] == 0


def test_density_box_matches_the_printed_closed_form(oracle):
    # Pressure is kept far from zero, so only the density box acts.
    A1 = prim_to_cons(np.array([0.5, 0, 0, 0, 0, 0, 0, 100.0]), G)
    H = np.zeros((4, 8))
    H[:, 0] = [-0.4, -0.3, 0.1, -0.2]
    lam, _ = oracle.flux_limiter_box(A1, H, G, 1e-13, 1e-13)
    expect = min(1.0, (0.5 - 1e-13) / (1e-12 + 0.9))
    np.testing.assert_allclose(lam, [expect, expect, 1.0, expect], rtol=1e-15)


def cubic_root(A1, D, g, eps_p):
    # rho(r) p(r)/(g-1) with A(r) = A1 + r D is a cubic in r; find its root in (0,1).
    rho = np.array([D[0], A1[0]])
    E = np.array([D[7], A1[7]])
    poly = np.polymul(rho, E)
    for q in (1, 2, 3):
        poly = np.polysub(poly, 0.5 * np.polymul([D[q], A1[q]], [D[q], A1[q]]))
    for q in (4, 5, 6):
        poly = np.polysub(poly, 0.5 * np.polymul(rho, np.polymul([D[q], A1[q]], [D[q], A1[q]])))
    poly = np.polysub(poly, rho * eps_p / (g - 1))
    roots = np.roots(poly)
    real = roots[np.abs(roots.imag) < 1e-9].real
    inside = real[(real > 0) & (real < 1)]
    return inside.min()


def test_vertex_root_matches_cubic_roots(oracle):
    iters = []
    for A1, H in cases(31, 200):
        D = H.sum(0)
        W = A1 + D
        if W[0] <= 0.05 * A1[0] or p_of(W) >= 1e-13:
            continue
        r, it = oracle.vertex_root(A1, D, G, 1e-13)
        iters.append(it)
        assert r == pytest.approx(cubic_root(A1, D, G, 1e-13), abs=1e-12)
        tol = 1e-14 * (np.max(np.abs(A1)) + np.max(np.abs(D))) ** 2
        assert p_of(A1 + r * D) == pytest.approx(1e-13, abs=tol)
    assert len(iters) > 10
    assert max(iters) <= 15, iters  # no bisection crawl: Newton converges


def test_point_scaling_limiter(oracle):
    rng = np.random.default_rng(41)
    n_active = 0
    for _ in range(400):
        wl = np.array([rng.uniform(0.1, 2), *rng.uniform(-1, 1, 6), rng.uniform(1e-3, 1)])
        UL = prim_to_cons(wl, G)
        UH = UL + rng.normal(size=8) * np.abs(UL) * 10 ** rng.uniform(-2, 0.7)
        out, nf = oracle.point_limiter(UH, UL, G)
        assert nf == 0
        er, ep = eps_of(UL)
        assert out[0] >= er * (1 - 1e-12) and p_of(out) >= ep * (1 - 1e-6) - 1e-15
        if UH[0] >= er and p_of(UH) >= ep:
            assert np.array_equal(out, UH)  # admissible input untouched
            continue
        n_active += 1
        # the result lies on the segment [Us, UL] where Us = UH with its density
        # blended: out - UL is parallel to (Us - UL) in the non-density part.
        d = UH[1:] - UL[1:]
        t = (out[1:] - UL[1:]) @ d / (d @ d)
        assert -1e-12 <= t <= 1 + 1e-12
        np.testing.assert_allclose(out[1:], UL[1:] + t * d, rtol=1e-9, atol=1e-12)
        # ... and is not more limited than the exact pressure-feasible blend
        lo, hi = 0.0, 1.0
        Us = UH.copy()
        if UH[0] < er:
            th1 = (UL[0] - er) / (UL[0] - UH[0])
            Us[0] = th1 * UH[0] + (1 - th1) * UL[0]
        f = lambda th: p_of(th * Us + (1 - th) * UL) - ep
        if f(1.0) < 0:
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if f(mid) >= 0 else (lo, mid)
            assert t <= hi + 1e-12
    assert n_active > 100


def test_source_limiter_step(oracle):
    # Step (1) of the flux limiter: the high-order source is blended with the
    # LLF source until p(A^{Lim,1}) >= eps_p; A^{Lim,1} lies on the segment
    # between the LLF state and the source-replaced state, no further from
    # the latter than the exact pressure-feasible blend.
    rng = np.random.default_rng(51)
    n_active = 0
    for _ in range(600):
        w = np.array([rng.uniform(0.3, 2), *rng.uniform(-1, 1, 6), rng.uniform(1e-3, 0.3)])
        A = prim_to_cons(w, G)
        Fl = rng.normal(size=(4, 8)) * 0.01
        Fs = Fl + rng.normal(size=(4, 8)) * 0.01
        S_llf = rng.normal(size=8) * 0.01
        S_llf[0] = 0.0
        S_s = S_llf + rng.normal(size=8) * 10 ** rng.uniform(-1, 1.5)
        S_s[0] = 0.0
        dt, dx, dy = 0.05, 0.7, 0.9
        th, lam, A1, nf = oracle.cell_limiter(A, Fs, Fl, S_s, S_llf, dt, dx, dy, G)
        assert nf == 0 and 0 <= th <= 1 and np.all((0 <= lam) & (lam <= 1))
        G_ = A - dt / dx * (Fl[1] - Fl[0]) - dt / dy * (Fl[3] - Fl[2])
        Allf, Asrc = G_ - dt * S_llf, G_ - dt * S_s
        np.testing.assert_allclose(A1, th * Asrc + (1 - th) * Allf, rtol=1e-12, atol=1e-12)
        ep = min(1e-13, p_of(Allf))
        if p_of(Asrc) >= ep:
            assert th == 1.0
            continue
        n_active += 1
        assert p_of(A1) >= ep - 1e-14 * np.abs(A1).max() ** 2
        lo, hi = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if p_of(mid * Asrc + (1 - mid) * Allf) >= ep else (lo, mid)
        assert th <= hi + 1e-12
    assert n_active > 50
