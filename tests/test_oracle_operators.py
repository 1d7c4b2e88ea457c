"""Pins of the oracle's discrete operators (Section 2.1-2.3, Section 3.4):
exactness on polynomials, closed-form values of the shock sensor."""
import math
from dataclasses import replace

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I
from paper_2506_04857_amd.inputs import OUTFLOW, PERIODIC, Problem, prim_to_cons


# ---------------------------------------------------------------- FVS (2d_fd)
def line_states(g, s, p_of_s, rho=1.3, v=(0.4, -0.3, 0.2)):
    ws = [np.array([rho, *v, 0.0, 0.0, 0.0, p_of_s(si)]) for si in s]
    return np.stack([prim_to_cons(w, g) for w in ws])


@pytest.mark.parametrize("d", [0, 1])
def test_fvs_exact_when_flux_is_quadratic_along_the_line(oracle, d):
    # B = 0, rho and v constant, p quadratic: F and U are quadratic in s, the
    # one-sided operators D+- are exact and the alpha terms cancel, so
    # D+F+ + D-F- equals the exact derivative (F(h/2) - F(-h/2)) / h.
    g, h = 5 / 3, 0.37
    p = lambda s: 1.0 + 0.8 * s - 1.7 * s * s
    s = np.array([-h, -h / 2, 0.0, h / 2, h])
    w = line_states(g, s, p)
    R, _ = oracle.fvs_derivative(w, g, d, h)
    ends = line_states(g, np.array([-h / 2, h / 2]), p)
    exact = (oracle.flux(ends[1], g, d) - oracle.flux(ends[0], g, d)) / h
    np.testing.assert_allclose(R, exact, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [0, 1])
def test_fvs_divergence_part_is_central_and_exact_on_parabolas(oracle, d):
    g, h = 1.4, 0.21
    s = np.array([-h, -h / 2, 0.0, h / 2, h])
    Bl = lambda t: 0.3 - 1.1 * t + 2.3 * t * t
    ws = []
    for si in s:
        B = [0.2, -0.1, 0.05]
        B[d] = Bl(si)
        ws.append(prim_to_cons(np.array([1.0, 0.1, 0.2, 0.0, *B, 2.0]), g))
    _, dB = oracle.fvs_derivative(np.stack(ws), g, d, h)
    assert dB == pytest.approx(-1.1, rel=1e-12)


def test_fvs_is_second_order_for_a_nonlinear_flux(oracle):
    g = 5 / 3
    def states(h):
        s = np.array([-h, -h / 2, 0.0, h / 2, h])
        out = []
        for si in s:
            w = np.array([1.0 + 0.3 * np.sin(si + 0.2), 0.5 * np.cos(si), 0.2, -0.1, 0.4 + 0.2 * np.sin(2 * si), 0.3,
                          0.1 * np.cos(si), 1.0 + 0.2 * np.sin(si)])
            out.append(prim_to_cons(w, g))
        return np.stack(out)
    def exact():
        e = 1e-5
        a = states(2 * e)
        return (oracle.flux(a[3], g, 0) - oracle.flux(a[1], g, 0)) / (2 * e)
    ex = exact()
    errs = []
    for h in (0.2, 0.1, 0.05):
        R, _ = oracle.fvs_derivative(states(h), g, 0, h)
        errs.append(np.max(np.abs(R - ex)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


# ------------------------------------------------ centre value and source
def poly_grid(nx, ny, coeffs, x0=0.1, y0=-0.3, L=1.0, bc=OUTFLOW):
    """State whose conservative components are bi-quadratic polynomials
    sum_{a,b<=2} c[q][a][b] x^a y^b, with exact cell averages."""
    prob = Problem("poly", nx, ny, x0, x0 + L, y0, y0 + L * ny / nx, 1.4, 0.2, 1.0, bc, bc, 1.0)
    dx, dy = prob.dx, prob.dy
    xe = x0 + np.arange(nx + 1) * dx
    ye = y0 + np.arange(ny + 1) * dy
    xn = x0 + np.arange(prob.nxp) * dx
    yn = y0 + np.arange(prob.nyp) * dy
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy

    def mono_avg(a, e):
        return (e[1:] ** (a + 1) - e[:-1] ** (a + 1)) / ((a + 1) * (e[1:] - e[:-1]))

    def evalp(c, X, Y):
        return sum(c[a][b] * X ** a * Y ** b for a in range(3) for b in range(3))

    cell = np.zeros((8, ny, nx))
    for q in range(8):
        for a in range(3):
            for b in range(3):
                cell[q] += coeffs[q][a][b] * np.outer(mono_avg(b, ye), mono_avg(a, xe))
    XX, YY = np.meshgrid(xn, yc)
    xface = np.stack([evalp(coeffs[q], XX, YY) for q in range(8)])
    XX, YY = np.meshgrid(xc, yn)
    yface = np.stack([evalp(coeffs[q], XX, YY) for q in range(8)])
    XX, YY = np.meshgrid(xn, yn)
    vert = np.stack([evalp(coeffs[q], XX, YY) for q in range(8)])
    XX, YY = np.meshgrid(xc, yc)
    centre = np.stack([evalp(coeffs[q], XX, YY) for q in range(8)])
    return prob, (cell, xface, yface, vert), centre, evalp


def test_centre_value_exact_on_biquadratics(oracle):
    rng = np.random.default_rng(11)
    c = rng.uniform(-0.3, 0.3, (8, 3, 3))
    c[0, 0, 0] = 2.0
    c[7, 0, 0] = 40.0
    prob, u, centre, _ = poly_grid(7, 5, c)
    C, _, _ = oracle.cell_diagnostics(prob, u)
    np.testing.assert_allclose(C, centre, rtol=1e-13, atol=1e-13)


def test_cell_source_vanishes_for_divergence_free_biquadratic_field(oracle):
    rng = np.random.default_rng(12)
    c = rng.uniform(-0.3, 0.3, (8, 3, 3))
    c[0, 0, 0] = 2.0
    c[7, 0, 0] = 40.0
    # B1 = y^2 + x y - x^2, B2 = x^2 + 2 x y - y^2/2 (+ constants): div B = 0
    c[4] = 0.0
    c[5] = 0.0
    c[4][0][2], c[4][1][1], c[4][2][0], c[4][0][0] = 1.0, 1.0, -1.0, 0.7
    c[5][2][0], c[5][1][1], c[5][0][2], c[5][0][0] = 1.0, 2.0, -0.5, -0.4
    prob, u, _, _ = poly_grid(6, 6, c)
    _, S, _ = oracle.cell_diagnostics(prob, u)
    assert np.max(np.abs(S)) < 1e-13


def test_cell_source_is_exact_average_of_divB_psi(oracle):
    # v = 0 so Psi = (0, B, 0, 0, 0, 0); B1 quadratic in x / linear in y, B2
    # linear in x / quadratic in y, B3 bi-quadratic: the nine-point divergence
    # is exact and (div B) B has degree <= 3 per variable, where the 3x3
    # Simpson rule is exact.  Reference: Gauss-Legendre 4x4 per cell.
    rng = np.random.default_rng(13)
    c = np.zeros((8, 3, 3))
    c[0, 0, 0] = 1.5
    c[7, 0, 0] = 30.0
    c[4][:, :2] = rng.uniform(-1, 1, (3, 2))
    c[5][:2, :] = rng.uniform(-1, 1, (2, 3))
    c[6] = rng.uniform(-1, 1, (3, 3))
    prob, u, _, evalp = poly_grid(5, 4, c)
    _, S, _ = oracle.cell_diagnostics(prob, u)
    gx, gw = np.polynomial.legendre.leggauss(4)

    def dpoly_x(cq, X, Y):
        return sum(a * cq[a][b] * X ** (a - 1) * Y ** b for a in range(1, 3) for b in range(3))

    def dpoly_y(cq, X, Y):
        return sum(b * cq[a][b] * X ** a * Y ** (b - 1) for a in range(3) for b in range(1, 3))

    for j in range(prob.ny):
        for i in range(prob.nx):
            xa, ya = prob.x0 + i * prob.dx, prob.y0 + j * prob.dy
            X, Y = np.meshgrid(xa + 0.5 * prob.dx * (gx + 1), ya + 0.5 * prob.dy * (gx + 1))
            W = 0.25 * np.outer(gw, gw)
            div = dpoly_x(c[4], X, Y) + dpoly_y(c[5], X, Y)
            for q in (1, 2, 3):
                expect = np.sum(W * div * evalp(c[3 + q], X, Y))
                assert S[q, j, i] == pytest.approx(expect, rel=1e-11, abs=1e-12)
            assert np.all(S[[0, 4, 5, 6, 7], j, i] == 0.0)


def test_simpson_flux_exact_on_cubic_edge_profile(oracle):
    # B = 0, rho, v constant, p cubic in y along the edge: F1 is linear in p,
    # so the Simpson flux is the exact edge average v1 U(pbar) + pbar (e1 + v1 e7).
    g = 5 / 3
    nx = ny = 4
    prob = Problem("edge", nx, ny, 0.0, 1.0, 0.0, 1.0, g, 0.2, 1.0, PERIODIC, PERIODIC, 1.0)
    p = lambda y: 1.0 + 0.5 * y - 0.7 * y ** 2 + 0.9 * y ** 3
    pint = lambda y: y + 0.25 * y ** 2 - 0.7 / 3 * y ** 3 + 0.225 * y ** 4
    v1 = 0.6

    def cons(pv):
        return prim_to_cons(np.array([1.2, v1, 0.0, 0.0, 0.0, 0.0, 0.0, pv]), g)

    state = []
    for shape, ys in (((8, ny, nx), (np.arange(ny) + 0.5) / ny), ((8, ny, nx), (np.arange(ny) + 0.5) / ny),
                      ((8, ny, nx), np.arange(ny) / ny), ((8, ny, nx), np.arange(ny) / ny)):
        a = np.zeros(shape)
        for jj, y in enumerate(ys):
            a[:, jj, :] = cons(p(y))[:, None]
        state.append(a)
    j = 1
    F = oracle.simpson(prob, tuple(state), 0, 2, j)
    pbar = (pint((j + 1) / ny) - pint(j / ny)) * ny
    e = np.zeros(8)
    e[1], e[7] = 1.0, v1
    np.testing.assert_allclose(F, v1 * cons(pbar) + pbar * e, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------ shock sensor
def cell_field_problem(nx, ny, prim_cell, g=5 / 3):
    prob = Problem("s", nx, ny, 0.0, 1.0, 0.0, ny / nx, g, 0.2, 1.0, PERIODIC, PERIODIC, 1.0)
    xc = (np.arange(nx) + 0.5) * prob.dx
    yc = (np.arange(ny) + 0.5) * prob.dy
    X, Y = np.meshgrid(xc, yc)
    cell = prim_to_cons(prim_cell(X, Y), g)
    pts = [np.zeros(s) for s in prob.shapes()[1:]]
    for a in pts:
        a[...] = cell.mean(axis=(1, 2))[:, None, None]
    return prob, (cell, *pts)


def test_sensor_closed_forms(oracle):
    one = lambda X: np.ones_like(X)
    # constant state: all three indicators vanish
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), 0.3 * one(X), 0.1 * one(X), 0 * X, 0.5 * one(X),
                                                            0.2 * one(X), 0 * X, one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    assert np.max(np.abs(s)) < 1e-15
    # rigid rotation v = (-y', x') about a cell centre: div v = 0 -> phi2 = 0
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), -(Y - 0.5625), X - 0.5625, 0 * X, 0 * X, 0 * X,
                                                            0 * X, 2 * one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    assert np.max(np.abs(s[2, 2:6, 2:6])) < 1e-13
    # uniform compression v = -(x', y'): div < 0, curl = 0 -> phi2 = 1
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), -(X - 0.5), -(Y - 0.5), 0 * X, 0 * X, 0 * X,
                                                            0 * X, 2 * one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    np.testing.assert_allclose(s[2, 2:6, 2:6], 1.0, rtol=1e-13)
    # compression with rotation v = (-x' - y', x' - y'): div = -2, curl = 2, phi2 = 2/sqrt(8)
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), -(X - 0.5) - (Y - 0.5), (X - 0.5) - (Y - 0.5),
                                                            0 * X, 0 * X, 0 * X, 0 * X, 2 * one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    np.testing.assert_allclose(s[2, 2:6, 2:6], 2 / np.sqrt(8), rtol=1e-13)
    # expansion: phi2 = 0
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), X - 0.5, Y - 0.5, 0 * X, 0 * X, 0 * X, 0 * X,
                                                            2 * one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    assert np.max(np.abs(s[2, 2:6, 2:6])) == 0.0
    # B1 = x + 3 (div B = 1), B2 = 0: phi3 = (B1(i+1) - B1(i-1)) / |B1 + B2| = 2 dx / (x_i + 3)
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), 0 * X, 0 * X, 0 * X, X + 3.0, 0 * X, 0 * X,
                                                            20 * one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    xc = (np.arange(8) + 0.5) / 8
    np.testing.assert_allclose(s[3, :, 2:6], (2 * prob.dx / (xc + 3.0))[None, 2:6].repeat(8, 0), rtol=1e-12)
    # divergence-free B = (f(y), g(x)): phi3 = 0
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), 0 * X, 0 * X, 0 * X, np.sin(2 * np.pi * Y) + 2,
                                                            np.cos(2 * np.pi * X), 0 * X, 20 * one(X)]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    assert np.max(s[3]) < 1e-14
    # total pressure linear in x: phi1x = 0; quadratic: known ratio
    prob, u = cell_field_problem(8, 8, lambda X, Y: np.stack([one(X), 0 * X, 0 * X, 0 * X, 0 * X, 0 * X, 0 * X,
                                                            1.0 + X ** 2]))
    _, _, s = oracle.cell_diagnostics(prob, u)
    xc = (np.arange(8) + 0.5) / 8
    dx = 1 / 8
    expect = (2 * dx * dx) / (4 * (1 + xc ** 2) + 2 * dx * dx)
    np.testing.assert_allclose(s[0, :, 1:7], expect[None, 1:7].repeat(8, 0), rtol=1e-11)
    assert np.max(np.abs(s[1])) < 1e-15


def _linear_field_state(prob, b1, b2):
    """A state with rho = 1, v = 0, p = 1 and B = (b1(x, y), b2(x, y), 0)
    sampled at every DoF (cell averages: the centre value suffices for the
    linear fields used here, whose averages equal their centre values)."""
    def prim(x, y, t):
        one = np.ones_like(x)
        return np.stack([one, 0 * one, 0 * one, 0 * one, b1(x, y) * one, b2(x, y) * one, 0 * one, one])
    return I.sample(replace(prob, prim=prim))


def test_divb_diagnostics_vanish_for_divergence_free_fields(oracle):
    # B = (y^2 - y, x^2 - x) (each component independent of its own
    # direction): both discrete divergences vanish to rounding.
    prob = replace(I.constant_state(12, bc=I.OUTFLOW), nx=12, ny=10)
    u = _linear_field_state(prob, lambda x, y: y * y - y, lambda x, y: x * x - x)
    d1, d2 = oracle.divb(prob, u)
    assert d1 < 1e-12 and d2 < 1e-12


def test_divb_diagnostics_exact_for_a_linear_field(oracle):
    # B1 = x, B2 = 0: div B = 1 everywhere, and the one-sided / central
    # differences of each cell are exact on linear data, so div1 is the
    # domain's area; the printed Gauss-Green form gives, per cell,
    # (1/6) |6 dx| dx dy, i.e. div2 = dx * area.
    prob = replace(I.constant_state(12, bc=I.OUTFLOW), nx=12, ny=10, x1=1.5, y1=2.0)
    u = _linear_field_state(prob, lambda x, y: x, lambda x, y: 0 * x)
    d1, d2 = oracle.divb(prob, u)
    area = (prob.x1 - prob.x0) * (prob.y1 - prob.y0)
    assert d1 == pytest.approx(area, rel=1e-13)
    assert d2 == pytest.approx(prob.dx * area, rel=1e-13)
    # the y-direction counterpart
    u = _linear_field_state(prob, lambda x, y: 0 * x, lambda x, y: -2 * y)
    d1, d2 = oracle.divb(prob, u)
    assert d1 == pytest.approx(2 * area, rel=1e-13)
    assert d2 == pytest.approx(2 * prob.dy * area, rel=1e-13)
