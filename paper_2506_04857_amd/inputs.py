"""Seeded, synthetic inputs: problem set-ups and initial data.

This module holds no arithmetic of the numerical method.  It describes each
workload (grid, domain, boundary conditions, gamma, CFL, shock-sensor kappa,
final time) and samples the initial data: cell averages by a 5x5
Gauss-Legendre rule per cell, point values by evaluation at the degree-of-
freedom locations.  Conservative variables are U = (rho, rho v, B, E) with
E = p/(gamma-1) + rho |v|^2 / 2 + |B|^2 / 2 (Section 1 of the paper).

A state is a tuple ``(cell, xface, yface, vert)`` of float64 arrays of shapes
``(8, ny, nx)``, ``(8, ny, nxp)``, ``(8, nyp, nx)``, ``(8, nyp, nxp)``, where
``nxp = nx`` for a periodic x direction and ``nx + 1`` for outflow (likewise y):
  cell[c, j, i]   average over cell (i, j)
  xface[c, j, k]  value at (x_{k-1/2}, y_j)
  yface[c, l, i]  value at (x_i, y_{l-1/2})
  vert[c, l, k]   value at (x_{k-1/2}, y_{l-1/2})
Both the HIP library and the CPU oracle consume these arrays; neither is
imported here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Callable

import numpy as np

PERIODIC, OUTFLOW = 0, 1
BASE_SEED = 2506


@dataclass(frozen=True)
class Problem:
    name: str
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    gamma: float
    cfl: float = 0.2
    kappa: float = 1.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    t_final: float = 1.0
    # primitive initial data: f(x, y, t) -> (rho, v1, v2, v3, B1, B2, B3, p)
    prim: Callable | None = field(default=None, compare=False, repr=False)

    @property
    def nxp(self) -> int:
        return self.nx + (1 if self.bc_x == OUTFLOW else 0)

    @property
    def nyp(self) -> int:
        return self.ny + (1 if self.bc_y == OUTFLOW else 0)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny

    def with_size(self, nx: int, ny: int | None = None) -> "Problem":
        return replace(self, nx=nx, ny=nx if ny is None else ny)

    def shapes(self):
        return ((8, self.ny, self.nx), (8, self.ny, self.nxp), (8, self.nyp, self.nx), (8, self.nyp, self.nxp))

    def cells(self) -> int:
        return self.nx * self.ny


def prim_to_cons(w: np.ndarray, gamma: float) -> np.ndarray:
    """(rho, v1, v2, v3, B1, B2, B3, p) -> (rho, rho v, B, E); leading axis 8."""
    rho, v1, v2, v3, B1, B2, B3, p = w
    E = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3) + 0.5 * (B1 * B1 + B2 * B2 + B3 * B3)
    return np.stack([rho, rho * v1, rho * v2, rho * v3, B1, B2, B3, E])


_GL_X, _GL_W = np.polynomial.legendre.leggauss(5)


def sample(prob: Problem, t: float = 0.0, gl: int = 5):
    """Initial (or exact, where the set-up has one) state at time t; cell
    averages by a gl x gl Gauss-Legendre rule (5 unless stated)."""
    gx, gw = (_GL_X, _GL_W) if gl == 5 else np.polynomial.legendre.leggauss(gl)
    f = prob.prim
    g = prob.gamma
    dx, dy = prob.dx, prob.dy
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * dx
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * dy
    xn = prob.x0 + np.arange(prob.nxp) * dx
    yn = prob.y0 + np.arange(prob.nyp) * dy

    def cons_at(X, Y):
        return prim_to_cons(np.asarray(f(X, Y, t), dtype=np.float64) * np.ones_like(X), g)

    # cell averages: 5x5 Gauss-Legendre per cell
    cell = np.zeros((8, prob.ny, prob.nx))
    for a in range(gl):
        for b in range(gl):
            X, Y = np.meshgrid(xc + 0.5 * dx * gx[a], yc + 0.5 * dy * gx[b])
            cell += 0.25 * gw[a] * gw[b] * cons_at(X, Y)
    X, Y = np.meshgrid(xn, yc)
    xface = cons_at(X, Y)
    X, Y = np.meshgrid(xc, yn)
    yface = cons_at(X, Y)
    X, Y = np.meshgrid(xn, yn)
    vert = cons_at(X, Y)
    return tuple(np.ascontiguousarray(a) for a in (cell, xface, yface, vert))


def _stack(*comps):
    return np.stack(np.broadcast_arrays(*comps))


# ------------------------------------------------------------------ problems
def alfven(n: int = 32) -> Problem:
    """Circularly polarised Alfven wave along 45 degrees; exact solution
    phi = 2 pi (x cos a + y sin a + t): it returns to its initial state at t=1."""
    a = math.pi / 4
    ca, sa = math.cos(a), math.sin(a)

    def prim(x, y, t):
        phi = 2 * math.pi * (x * ca + y * sa + t)
        s, c = np.sin(phi), np.cos(phi)
        vpar, vperp, v3 = 0.0, 0.1 * s, 0.1 * c
        bpar, bperp, b3 = 1.0, 0.1 * s, 0.1 * c
        v1 = vpar * ca - vperp * sa
        v2 = vpar * sa + vperp * ca
        B1 = bpar * ca - bperp * sa
        B2 = bpar * sa + bperp * ca
        one = np.ones_like(x)
        return _stack(one, v1, v2, v3 * one, B1, B2, b3 * one, 0.1 * one)

    return Problem("alfven", n, n, 0.0, 1.0 / ca, 0.0, 1.0 / sa, 5.0 / 3.0, 0.2, 1.0, PERIODIC, PERIODIC, 1.0, prim)


def orszag_tang(n: int = 512) -> Problem:
    """Orszag-Tang vortex on [0, 2 pi]^2 (the paper's set-up rescaled)."""
    gm = 5.0 / 3.0

    def prim(x, y, t):
        one = np.ones_like(x)
        return _stack(gm * gm * one, -np.sin(y), np.sin(x), 0 * one, -np.sin(y), np.sin(2 * x), 0 * one, gm * one)

    return Problem("orszag_tang", n, n, 0.0, 2 * math.pi, 0.0, 2 * math.pi, gm, 0.2, 1.0, PERIODIC, PERIODIC,
                   math.pi, prim)


BATCH_SIZES = (64, 96, 128, 192, 256)


def batched_orszag_tang(count: int = 256, seed: int = BASE_SEED, sizes=BATCH_SIZES) -> list:
    """An ensemble of independent periodic Orszag-Tang problems: instance k
    has nx and ny drawn independently from sizes (generator seed), and each
    primitive field (rho, v1, v2, v3, B1, B2, B3, p) scaled by 1 + 0.05 z
    with z ~ N(0, 1) from its own generator (seed + 1 + k); v3 = B3 = 0 stay
    zero, p stays positive and div B stays zero."""
    rng = np.random.default_rng(seed)
    dims = rng.choice(np.asarray(sizes), size=(count, 2))
    out = []
    base = orszag_tang(int(dims[0][0]))
    for k in range(count):
        z = np.random.default_rng(seed + 1 + k).standard_normal(8)
        scale = 1.0 + 0.05 * z

        def prim(x, y, t, scale=scale):
            return base.prim(x, y, t) * scale.reshape(8, *([1] * np.ndim(x)))

        out.append(replace(base, name=f"orszag_tang_batch_{k}", nx=int(dims[k][0]), ny=int(dims[k][1]), prim=prim))
    return out


def orszag_tang_paper(n: int = 400) -> Problem:
    """Orszag-Tang vortex exactly as in the paper: [0,1]^2, T = 0.5."""
    def prim(x, y, t):
        one = np.ones_like(x)
        s4 = math.sqrt(4 * math.pi)
        return _stack(25 / (36 * math.pi) * one, -np.sin(2 * math.pi * y), np.sin(2 * math.pi * x), 0 * one,
                      -np.sin(2 * math.pi * y) / s4, np.sin(4 * math.pi * x) / s4, 0 * one, 5 / (12 * math.pi) * one)

    return Problem("orszag_tang_paper", n, n, 0.0, 1.0, 0.0, 1.0, 5.0 / 3.0, 0.2, 1.0, PERIODIC, PERIODIC, 0.5,
                   prim)


def blast_lowbeta(n: int = 1024) -> Problem:
    """Low-beta blast: [-0.5,0.5]^2, outflow, B = (100/sqrt(4 pi), 0, 0),
    p = 1000 inside r < 0.1, 0.1 outside, gamma = 1.4, T = 0.01."""
    b1 = 100.0 / math.sqrt(4 * math.pi)

    def prim(x, y, t):
        one = np.ones_like(x)
        r = np.sqrt(x * x + y * y)
        p = np.where(r < 0.1, 1000.0, 0.1)
        return _stack(one, 0 * one, 0 * one, 0 * one, b1 * one, 0 * one, 0 * one, p)

    return Problem("blast_lowbeta", n, n, -0.5, 0.5, -0.5, 0.5, 1.4, 0.2, 1.0, OUTFLOW, OUTFLOW, 0.01, prim)


def blast_paper(n: int = 400) -> Problem:
    """Blast of the paper: B = (1/sqrt2, 1/sqrt2, 0), p = 10 / 0.1, gamma 5/3, T = 0.2."""
    s = 1.0 / math.sqrt(2.0)

    def prim(x, y, t):
        one = np.ones_like(x)
        r = np.sqrt(x * x + y * y)
        p = np.where(r < 0.1, 10.0, 0.1)
        return _stack(one, 0 * one, 0 * one, 0 * one, s * one, s * one, 0 * one, p)

    return Problem("blast_paper", n, n, -0.5, 0.5, -0.5, 0.5, 5.0 / 3.0, 0.2, 1.0, OUTFLOW, OUTFLOW, 0.2, prim)


def sine_wave(n: int = 32) -> Problem:
    """Smooth sine wave of the 2D accuracy test; exact solution translates."""
    def prim(x, y, t):
        one = np.ones_like(x)
        return _stack(1 + 0.99 * np.sin(2 * math.pi * (x + y - 2 * t)), one, one, 0 * one, 0.1 * one, 0.1 * one,
                      0 * one, one)

    return Problem("sine_wave", n, n, 0.0, 1.0, 0.0, 1.0, 5.0 / 3.0, 0.2, 1.0, PERIODIC, PERIODIC, 0.1, prim)


def vortex(n: int = 32, mu: float = 5.389489439) -> Problem:
    """MHD vortex of the accuracy test, read with the 1/(2 pi) factors so that
    the central pressure is about 5.3e-12 for the printed mu; translates with
    the background velocity (1, 1)."""
    mu_h = mu / (2 * math.pi)
    xi_h = math.sqrt(2.0) * mu / (2 * math.pi)

    def prim(x, y, t):
        # periodic image of the translated vortex centre
        xs = np.mod(x - t + 10.0, 20.0) - 10.0
        ys = np.mod(y - t + 10.0, 20.0) - 10.0
        r2 = xs * xs + ys * ys
        e = np.exp(0.5 * (1 - r2))
        one = np.ones_like(x)
        dp = 0.5 * (mu_h ** 2 * (1 - r2) - xi_h ** 2) * np.exp(1 - r2)
        return _stack(one, 1 + xi_h * e * (-ys), 1 + xi_h * e * xs, 0 * one, mu_h * e * (-ys), mu_h * e * xs,
                      0 * one, 1 + dp)

    return Problem("vortex", n, n, -10.0, 10.0, -10.0, 10.0, 5.0 / 3.0, 0.2, 1.0, PERIODIC, PERIODIC, 0.1, prim)


def constant_state(n: int = 16, bc: int = PERIODIC, w=(1.3, 0.4, -0.7, 0.2, 0.9, -0.35, 0.5, 2.1)) -> Problem:
    def prim(x, y, t):
        one = np.ones_like(x)
        return _stack(*[c * one for c in w])

    return Problem("constant", n, n + 3, 0.0, 1.0, 0.0, 1.25, 5.0 / 3.0, 0.2, 1.0, bc, bc, 1.0, prim)


def random_smooth(n: int = 16, ny: int | None = None, seed: int = BASE_SEED, amp: float = 0.2, bc: int = PERIODIC,
                  gamma: float = 5.0 / 3.0, kappa: float = 1.0) -> Problem:
    """Seeded random trigonometric field around a positive mean state (for
    parity tests on ragged grids).  Not divergence free."""
    rng = np.random.default_rng(seed)
    base = np.array([1.0, 0.3, -0.2, 0.1, 0.6, -0.4, 0.3, 1.5])
    kx = rng.integers(1, 4, size=(8, 3))
    ky = rng.integers(1, 4, size=(8, 3))
    ph = rng.uniform(0, 2 * math.pi, size=(8, 3))
    am = rng.uniform(-1, 1, size=(8, 3)) * amp
    ny = n if ny is None else ny

    def prim(x, y, t):
        out = []
        for c in range(8):
            v = base[c] * np.ones_like(x)
            for q in range(3):
                v = v + am[c, q] * np.sin(2 * math.pi * (kx[c, q] * x + ky[c, q] * y) + ph[c, q])
            out.append(v)
        out[0] = np.abs(out[0]) + 0.2
        out[7] = np.abs(out[7]) + 0.2
        return _stack(*out)

    return Problem("random_smooth", n, ny, 0.0, 1.0, 0.0, ny / n, gamma, 0.2, kappa, bc, bc, 1.0, prim)


def random_shock(n: int = 16, ny: int | None = None, seed: int = BASE_SEED, bc: int = OUTFLOW,
                 field_jump: float = 0.0, centre: tuple | None = None) -> Problem:
    """Seeded random piecewise-constant states with a strong pressure and
    density jump across a random circle (limiter-active parity cases).  With
    field_jump > 0 the magnetic field also jumps across the circle, which
    makes div B nonzero there.  ``centre`` (in units of the x extent) places
    the circle, e.g. on a boundary so that the jump crosses it."""
    rng = np.random.default_rng(seed)
    ny = n if ny is None else ny
    cx, cy = rng.uniform(0.35, 0.65, size=2)
    if centre is not None:
        cx, cy = centre
    r0 = rng.uniform(0.15, 0.3)
    inner = np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]) + rng.uniform(-0.2, 0.2, size=8)
    inner[0], inner[7] = 1.0, 1000.0
    outer = np.array([0.1, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]) + rng.uniform(-0.2, 0.2, size=8)
    outer[0], outer[7] = 0.125, 1e-3
    b = rng.uniform(-5, 5, size=3)
    inner[4:7] = b
    outer[4:7] = b + field_jump * rng.uniform(-1, 1, size=3)

    def prim(x, y, t):
        r = np.sqrt((x - cx) ** 2 + (y * n / ny - cy) ** 2)
        ins = r < r0
        return _stack(*[np.where(ins, inner[c], outer[c]) for c in range(8)])

    return Problem("random_shock", n, ny, 0.0, 1.0, 0.0, ny / n, 1.4, 0.2, 1.0, bc, bc, 1.0, prim)


def low_beta_shock(n: int = 40, ny: int | None = None, seed: int = 3, b_mag: float = 1e4, p_in: float = 100.0,
                   p_out: float = 1e-4, bc: int = OUTFLOW) -> Problem:
    """Piecewise-constant data whose variables' scales differ a lot, as in
    the paper's jets: a uniform field of strength b_mag (|B|^2/2 = 5e7 at
    1e4) in a random direction, a disc of rho = 1, v = 0, p = p_in in a
    moving ambient of rho = 0.1, p = p_out.  The pressure of a limited
    state is then decided by the round-off of E - |m|^2/(2 rho) - |B|^2/2,
    and the round-off fallback of the closing remark of Section 4 acts."""
    rng = np.random.default_rng(seed)
    ny = n if ny is None else ny
    cx, cy = rng.uniform(0.35, 0.65, size=2)
    r0 = rng.uniform(0.15, 0.3)
    th = rng.uniform(0.0, 2.0 * math.pi)
    b1, b2 = b_mag * math.cos(th), b_mag * math.sin(th)
    v1, v2 = rng.uniform(-3.0, 3.0, size=2)

    def prim(x, y, t):
        ins = np.sqrt((x - cx) ** 2 + (y * n / ny - cy) ** 2) < r0
        z = np.zeros_like(np.asarray(x, dtype=np.float64))
        return _stack(np.where(ins, 1.0, 0.1), np.where(ins, 0.0, v1), np.where(ins, 0.0, v2), z, b1 + z, b2 + z, z,
                      np.where(ins, p_in, p_out))

    return Problem("low_beta_shock", n, ny, 0.0, 1.0, 0.0, ny / n, 1.4, 0.2, 1.0, bc, bc, 1.0, prim)


def stirred(base: Problem, eps: float = 1e-2) -> Problem:
    """base with a small smooth velocity field added (eps sin / cos waves in
    v1 and v2): the shock sensor's phi2 = -div v / |(div v, curl v)| is then
    differentiable everywhere, also in regions where base has a constant
    velocity (there div v and curl v are rounding noise and phi2 is 0/0)."""
    def prim(x, y, t):
        w = np.array(base.prim(x, y, t) * np.ones_like(np.asarray(x, dtype=np.float64)), dtype=np.float64)
        w[1] = w[1] + eps * np.sin(2 * math.pi * (x + 2 * y) + 0.3)
        w[2] = w[2] + eps * np.cos(2 * math.pi * (2 * x - y) + 1.1)
        return w

    return replace(base, name=base.name + "_stirred", prim=prim)


ADJOINT_STEPS = 400


def alfven_perturbed(n: int = 256, seed: int = BASE_SEED + 999, amp: float = 1e-3) -> Problem:
    """The Alfven wave of ``alfven`` plus a seeded smooth perturbation of
    amplitude ``amp`` in rho and B1 (the adjoint workload, 256^2 by default).

    drho = amp * s / max|s| with s = sum_q a_q sin(2 pi (m_q x + n_q y)/L + psi_q),
    dB1  = amp * t / max|t| with t = sum_q b_q sin(2 pi n'_q y / L + chi_q),
    q = 1..3, L = sqrt(2) (the side of the domain), m, n, n' drawn from {1,2,3},
    a, b ~ N(0,1), phases ~ U[0, 2 pi), all from default_rng(seed) in that
    order; the maxima are taken on a 512 x 512 lattice of the periodic domain.
    dB1 depends on y only, so div B stays zero; p and the other primitives
    are those of the wave, and the conservative variables are recomputed."""
    base = alfven(n)
    L = base.x1 - base.x0
    rng = np.random.default_rng(seed)
    m = rng.integers(1, 4, size=3)
    nn = rng.integers(1, 4, size=3)
    a = rng.standard_normal(3)
    psi = rng.uniform(0.0, 2 * math.pi, size=3)
    nb = rng.integers(1, 4, size=3)
    b = rng.standard_normal(3)
    chi = rng.uniform(0.0, 2 * math.pi, size=3)

    def s_rho(x, y):
        return sum(a[q] * np.sin(2 * math.pi * (m[q] * x + nn[q] * y) / L + psi[q]) for q in range(3))

    def s_b1(y):
        return sum(b[q] * np.sin(2 * math.pi * nb[q] * y / L + chi[q]) for q in range(3))

    lat = np.arange(512) * (L / 512)
    X, Y = np.meshgrid(lat, lat)
    norm_rho = amp / np.max(np.abs(s_rho(X, Y)))
    norm_b1 = amp / np.max(np.abs(s_b1(lat)))

    def prim(x, y, t):
        w = base.prim(x, y, t)
        w = np.array(w * np.ones_like(np.asarray(x, dtype=np.float64)), dtype=np.float64)
        w[0] = w[0] + norm_rho * s_rho(x, y)
        w[4] = w[4] + norm_b1 * s_b1(y)
        return w

    return replace(base, name="alfven_perturbed", prim=prim)


def adjoint_objective_target(prob: Problem) -> float:
    """rho_target of J = 1/2 sum_cells (rho(T) - rho_target)^2: the density of
    the unperturbed wave, which is 1 everywhere at every time."""
    return 1.0


def adjoint_directions(prob: Problem, count: int = 20, seed: int = BASE_SEED + 1000) -> list:
    """Unit-Gaussian directions over all 32 planes of the initial state for
    the finite-difference check: direction k from default_rng(seed + k)."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(seed + k)
        out.append(tuple(rng.standard_normal(s) for s in prob.shapes()))
    return out


CONFIGS = {
    "alfven_32": lambda: alfven(32),
    "orszag_tang_512": lambda: orszag_tang(512),
    "blast_lowbeta_1024": lambda: blast_lowbeta(1024),
    "alfven_perturbed_256": lambda: alfven_perturbed(256),
}
