"""Pins of the oracle's physics building blocks (Section 1, eq. (cf), Lemma of
Section 3.1) against facts that do not come from the oracle itself."""
import numpy as np
import pytest

from paper_2506_04857_amd.inputs import prim_to_cons

GAMMAS = (5.0 / 3.0, 1.4, 2.0)


def random_states(rng, n, low_p=False):
    w = np.empty((n, 8))
    w[:, 0] = 10 ** rng.uniform(-2, 0.5, n) if low_p else rng.uniform(0.3, 3.0, n)
    w[:, 1:4] = rng.uniform(-2, 2, (n, 3))
    w[:, 4:7] = rng.uniform(-3, 3, (n, 3))
    w[:, 7] = 10 ** rng.uniform(-6, -1, n) if low_p else rng.uniform(0.05, 3.0, n)
    return w


def test_pressure_recovers_primitive(oracle):
    rng = np.random.default_rng(1)
    for g in GAMMAS:
        for w in random_states(rng, 50):
            U = prim_to_cons(w, g)
            assert oracle.pressure(U, g) == pytest.approx(w[7], rel=1e-12, abs=1e-13)


def swap(U):
    """x <-> y reflection of a conservative state."""
    return U[[0, 2, 1, 3, 5, 4, 6, 7]]


def test_flux_xy_symmetry(oracle):
    rng = np.random.default_rng(2)
    for w in random_states(rng, 40):
        U = prim_to_cons(w, 5 / 3)
        F1 = oracle.flux(U, 5 / 3, 0)
        F2 = oracle.flux(swap(U), 5 / 3, 1)
        np.testing.assert_allclose(swap(F2), F1, rtol=1e-13, atol=1e-13)


def test_flux_splits_into_advection_pressure_and_maxwell_stress(oracle):
    # F_l(U) = v_l U + p_t (e_{m_l} + v_l e_E) - B_l (0, B, v, v.B): the physical
    # flux regrouped as transport, total pressure and magnetic tension.
    rng = np.random.default_rng(3)
    for g in GAMMAS:
        for w in random_states(rng, 30):
            U = prim_to_cons(w, g)
            rho, v, B, p = w[0], w[1:4], w[4:7], w[7]
            pt = p + 0.5 * B @ B
            for d in (0, 1):
                e = np.zeros(8)
                e[1 + d] = 1.0
                e[7] = v[d]
                maxwell = np.concatenate([[0.0], B, v, [v @ B]])
                expect = v[d] * U + pt * e - B[d] * maxwell
                np.testing.assert_allclose(oracle.flux(U, g, d), expect, rtol=1e-11, atol=1e-11)
                assert oracle.flux(U, g, d)[4 + d] == 0.0


def numerical_jacobian(oracle, U, g, d, h=1e-6):
    J = np.zeros((8, 8))
    for q in range(8):
        e = np.zeros(8)
        e[q] = h * max(1.0, abs(U[q]))
        J[:, q] = (oracle.flux(U + e, g, d) - oracle.flux(U - e, g, d)) / (2 * e[q])
    return J


def test_spectral_radius_is_max_eigenvalue_of_flux_jacobian(oracle):
    # "One can verify that rho_l = |v_l| + c_{f,l}" (Section 2.3).
    rng = np.random.default_rng(4)
    for g in GAMMAS:
        for w in random_states(rng, 25):
            U = prim_to_cons(w, g)
            for d in (0, 1):
                lam = np.linalg.eigvals(numerical_jacobian(oracle, U, g, d))
                assert np.max(np.abs(lam)) == pytest.approx(oracle.spectral_radius(U, g, d), rel=2e-6)


def test_fast_speed_special_cases(oracle):
    g = 5 / 3
    # B = 0: fast speed is the sound speed
    w = np.array([1.7, 0.3, -0.2, 0.1, 0.0, 0.0, 0.0, 0.9])
    assert oracle.fast_speed(prim_to_cons(w, g), g, 0) == pytest.approx(np.sqrt(g * 0.9 / 1.7), rel=1e-14)
    # B_l = 0: c_f = sqrt(c^2 + |B|^2/rho) (perpendicular propagation)
    w = np.array([1.7, 0.3, -0.2, 0.1, 0.0, 0.8, -0.6, 0.9])
    expect = np.sqrt(g * 0.9 / 1.7 + 1.0 / 1.7)
    assert oracle.fast_speed(prim_to_cons(w, g), g, 0) == pytest.approx(expect, rel=1e-14)
    # field along l: c_f = max(c, c_A)
    w = np.array([1.7, 0.3, -0.2, 0.1, 0.0, 2.0, 0.0, 0.9])
    expect = max(np.sqrt(g * 0.9 / 1.7), 2.0 / np.sqrt(1.7))
    assert oracle.fast_speed(prim_to_cons(w, g), g, 1) == pytest.approx(expect, rel=1e-13)


def test_llf_flux_consistency_and_viscosity(oracle):
    rng = np.random.default_rng(5)
    g = 5 / 3
    ws = random_states(rng, 40)
    for a, b in zip(ws[::2], ws[1::2]):
        Ua, Ub = prim_to_cons(a, g), prim_to_cons(b, g)
        for d in (0, 1):
            # consistency F^LLF(U, U) = F(U); alpha(U, U) is the spectral radius
            np.testing.assert_allclose(oracle.llf_flux(Ua, Ua, g, d), oracle.flux(Ua, g, d), rtol=1e-14, atol=1e-14)
            assert oracle.alpha_llf(Ua, Ua, g, d) == pytest.approx(oracle.spectral_radius(Ua, g, d), rel=1e-14)
            al = oracle.alpha_llf(Ua, Ub, g, d)
            assert al >= oracle.spectral_radius(Ua, g, d) and al >= oracle.spectral_radius(Ub, g, d)
            assert al == oracle.alpha_llf(Ub, Ua, g, d)
            # conservation form: flux difference of the LLF flux from its definition
            F = oracle.llf_flux(Ua, Ub, g, d)
            np.testing.assert_allclose(
                F, 0.5 * (oracle.flux(Ua, g, d) + oracle.flux(Ub, g, d)) - 0.5 * al * (Ub - Ua), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("low_p", [False, True])
def test_point_llf_is_positivity_preserving_under_lemma_cfl(oracle, low_p):
    # Lemma (Wu): with alpha from the Lemma and dt under its CFL condition the
    # first-order LLF update with the central Powell source stays in G.
    rng = np.random.default_rng(6 + low_p)
    g, dx, dy = 1.4, 0.7, 1.3
    fails = 0
    for _ in range(3000):
        ws = random_states(rng, 5, low_p=low_p)
        U, L, R, D, Up = (prim_to_cons(w, g) for w in ws)
        aL = oracle.alpha_llf(L, U, g, 0)
        aR = oracle.alpha_llf(U, R, g, 0)
        aD = oracle.alpha_llf(D, U, g, 1)
        aU = oracle.alpha_llf(U, Up, g, 1)
        divB = (R[4] - L[4]) / (2 * dx) + (Up[5] - D[5]) / (2 * dy)
        bound = aL / dx + aR / dx + aD / dy + aU / dy + abs(divB) / np.sqrt(U[0])
        dt = 0.999 / bound
        W = oracle.point_llf(U, L, R, D, Up, dt, dx, dy, g)
        if not (W[0] > 0 and oracle.pressure(W, g) > 0):
            fails += 1
    assert fails == 0


def test_point_llf_breaks_beyond_cfl_somewhere(oracle):
    # Sanity of the previous pin: far beyond the CFL bound positivity is lost
    # for some draws, so the bound is what keeps the update admissible.
    rng = np.random.default_rng(8)
    g, dx, dy = 1.4, 0.7, 1.3
    bad = 0
    for _ in range(300):
        ws = random_states(rng, 5, low_p=True)
        U, L, R, D, Up = (prim_to_cons(w, g) for w in ws)
        W = oracle.point_llf(U, L, R, D, Up, 5.0, dx, dy, g)
        bad += not (W[0] > 0 and oracle.pressure(W, g) > 0)
    assert bad > 0

