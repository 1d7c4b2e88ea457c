"""Consistency pins: with a tiny time step (limiters inactive) the oracle's
forward-Euler stage recovers the semi-discrete right-hand sides of the point
values and cell averages, which must converge to the right-hand side of the
Godunov-Powell system, eq. (2d_mhd_gp),
    U_t = -(F1)_x - (F2)_y - (div B) Psi,
evaluated from the exact initial data.  A wrong sign, a dropped term, a
misplaced stencil point or a swapped direction anywhere in the update gives
an O(1) error and fails the convergence rate."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2506_04857_amd import inputs as I


def np_flux(U, g, d):
    # physical flux written as transport + total pressure + magnetic tension
    # (this regrouping is itself pinned against the oracle's flux)
    rho, m, B, E = U[0], U[1:4], U[4:7], U[7]
    v = m / rho
    p = (g - 1) * (E - 0.5 * (m * m).sum(0) / rho - 0.5 * (B * B).sum(0))
    pt = p + 0.5 * (B * B).sum(0)
    vB = (v * B).sum(0)
    F = v[d] * U
    F[1 + d] += pt
    F[7] += pt * v[d]
    psi = np.concatenate([np.zeros_like(rho)[None], B, v, vB[None]])
    return F - B[d] * psi


def exact_rhs(prob, X, Y):
    g = prob.gamma
    cons = lambda x, y: I.prim_to_cons(np.asarray(prob.prim(x, y, 0.0)) * np.ones_like(x), g)
    h = 1e-3

    def ddx(f, d):
        e = (h, 0.0) if d == 0 else (0.0, h)
        return (-f(X + 2 * e[0], Y + 2 * e[1]) + 8 * f(X + e[0], Y + e[1]) - 8 * f(X - e[0], Y - e[1])
                + f(X - 2 * e[0], Y - 2 * e[1])) / (12 * h)

    U = cons(X, Y)
    dF1 = ddx(lambda x, y: np_flux(cons(x, y), g, 0), 0)
    dF2 = ddx(lambda x, y: np_flux(cons(x, y), g, 1), 1)
    divB = ddx(lambda x, y: cons(x, y)[4], 0) + ddx(lambda x, y: cons(x, y)[5], 1)
    v = U[1:4] / U[0]
    psi = np.concatenate([np.zeros_like(U[0])[None], U[4:7], v, (v * U[4:7]).sum(0)[None]])
    return -dF1 - dF2 - divB * psi


def exact_rhs_state(prob):
    dx, dy = prob.dx, prob.dy
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * dx
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * dy
    xn = prob.x0 + np.arange(prob.nxp) * dx
    yn = prob.y0 + np.arange(prob.nyp) * dy
    gx, gw = np.polynomial.legendre.leggauss(5)
    cell = 0.0
    for a in range(5):
        for b in range(5):
            X, Y = np.meshgrid(xc + 0.5 * dx * gx[a], yc + 0.5 * dy * gx[b])
            cell = cell + 0.25 * gw[a] * gw[b] * exact_rhs(prob, X, Y)
    return (cell, exact_rhs(prob, *np.meshgrid(xn, yc)), exact_rhs(prob, *np.meshgrid(xc, yn)),
            exact_rhs(prob, *np.meshgrid(xn, yn)))


def discrete_rhs(oracle, prob, dt=1e-9):
    u = I.sample(prob)
    c = oracle.Counters()
    fe = oracle.stage(prob, 0, u, u, dt, counters=c)
    assert c.n_point_limited == 0 and c.n_theta_active == 0 and c.n_source_limited == 0
    return tuple((a - b) / dt for a, b in zip(fe, u))


def errors(oracle, kappa, sizes=(32, 64)):
    out = []
    for n in sizes:
        p = replace(I.random_smooth(n, n, seed=7, amp=0.1), kappa=kappa)
        num, ex = discrete_rhs(oracle, p), exact_rhs_state(p)
        out.append([np.max(np.abs(a - b)) for a, b in zip(num, ex)])
    return np.array(out)


def test_point_values_consistent_with_godunov_powell_system(oracle):
    e = errors(oracle, 1.0)
    rates = np.log2(e[0, 1:] / e[1, 1:])  # X, Y, V
    assert np.all(rates > 1.7), (e, rates)


def test_cell_averages_high_order_consistent(oracle):
    # kappa = 0: the shock sensor keeps the high-order Simpson flux and the
    # nine-point source.
    e = errors(oracle, 0.0)
    rate = np.log2(e[0, 0] / e[1, 0])
    assert rate > 3.0, (e[:, 0], rate)


def test_cell_averages_first_order_llf_when_sensor_saturates(oracle):
    # kappa -> infinity: every interface coefficient is exp(-inf) = 0 (the
    # data are not divergence free, so phi3 > 0), and the cell update is the
    # first-order LLF scheme of eq. (2d_llf): first-order consistent.
    e = errors(oracle, 1e300)
    rate = np.log2(e[0, 0] / e[1, 0])
    assert 0.7 < rate < 1.5, (e[:, 0], rate)
    e0 = errors(oracle, 0.0, sizes=(32,))
    assert e[0, 0] > 5 * e0[0, 0]  # the saturated sensor really switched to LLF
