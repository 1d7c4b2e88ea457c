"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path (the HIP library and
its binding) never imports or calls it.

A state is a tuple of four float64 arrays ``(cell, xface, yface, vert)`` with
shapes ``(8, ny, nx)``, ``(8, ny, nxp)``, ``(8, nyp, nx)``, ``(8, nyp, nxp)``
(``nxp = nx`` for a periodic x direction, ``nx + 1`` for outflow; same for y).
A problem is any object with the attributes ``nx, ny, x0, x1, y0, y1, gamma,
cfl, kappa, bc_x, bc_y`` (0 periodic, 1 outflow).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "af_oracle.cpp")
LIB = os.environ.get("AF_ORACLE_LIB") or os.path.join(HERE, "_build", "liboracle.so")
# The same source built on forward-mode dual numbers (-DORC_TANGENT=TANGENT_ND):
# exact directional derivatives of the discrete stage, the adjoint's reference.
TANGENT_ND = 8
TLIB = os.path.join(HERE, "_build", "liboracle_tangent.so")

# -O2 without -march=native: the library is built here and may run on another host.
CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def _compile(out: str, extra: list) -> None:
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", *CXXFLAGS, *extra, SRC, "-o", tmp])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/_build/liboracle.so`` and its tangent
    build into ``oracle/_build/liboracle_tangent.so``."""
    for out, extra in ((LIB, []), (TLIB, ["-DORC_TANGENT=%d" % TANGENT_ND])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            _compile(out, extra)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("kappa", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("nthreads", ctypes.c_int32),
    ]


class _Counters(ctypes.Structure):
    _fields_ = [
        ("n_llf_not_admissible", ctypes.c_int64), ("n_newton", ctypes.c_int64),
        ("newton_iters_max", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
        ("n_not_admissible", ctypes.c_int64), ("n_theta_active", ctypes.c_int64),
        ("n_point_limited", ctypes.c_int64), ("n_centre_limited", ctypes.c_int64),
        ("n_source_limited", ctypes.c_int64), ("min_theta", ctypes.c_double),
    ]


@dataclass
class Counters:
    n_llf_not_admissible: int = 0
    n_newton: int = 0
    newton_iters_max: int = 0
    n_fallback: int = 0
    n_not_admissible: int = 0
    n_theta_active: int = 0
    n_point_limited: int = 0
    n_centre_limited: int = 0
    n_source_limited: int = 0
    min_theta: float = 1.0

    def add(self, c: _Counters) -> None:
        self.n_llf_not_admissible += c.n_llf_not_admissible
        self.n_newton += c.n_newton
        self.newton_iters_max = max(self.newton_iters_max, c.newton_iters_max)
        self.n_fallback += c.n_fallback
        self.n_not_admissible += c.n_not_admissible
        self.n_theta_active += c.n_theta_active
        self.n_point_limited += c.n_point_limited
        self.n_centre_limited += c.n_centre_limited
        self.n_source_limited += c.n_source_limited
        self.min_theta = min(self.min_theta, c.min_theta)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_DD = ctypes.POINTER(_D)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_stage.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _DD, _DD, _DD, ctypes.c_double,
                                ctypes.POINTER(_Counters)]
        L.orc_stage.restype = ctypes.c_int
        L.orc_dt.argtypes = [ctypes.POINTER(_Params), _DD, ctypes.c_double]
        L.orc_dt.restype = ctypes.c_double
        L.orc_step.argtypes = [ctypes.POINTER(_Params), _DD, ctypes.c_double, ctypes.c_int, _D,
                               ctypes.POINTER(_Counters)]
        L.orc_step.restype = ctypes.c_int
        L.orc_pressure.argtypes = [_D, ctypes.c_double]
        L.orc_pressure.restype = ctypes.c_double
        L.orc_flux.argtypes = [_D, ctypes.c_double, ctypes.c_int, _D]
        L.orc_fast_speed.argtypes = [_D, ctypes.c_double, ctypes.c_int]
        L.orc_fast_speed.restype = ctypes.c_double
        L.orc_spectral_radius.argtypes = [_D, ctypes.c_double, ctypes.c_int]
        L.orc_spectral_radius.restype = ctypes.c_double
        L.orc_alpha_llf.argtypes = [_D, _D, ctypes.c_double, ctypes.c_int]
        L.orc_alpha_llf.restype = ctypes.c_double
        L.orc_llf_flux.argtypes = [_D, _D, ctypes.c_double, ctypes.c_int, _D]
        L.orc_fvs_derivative.argtypes = [_D, ctypes.c_double, ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_point_limiter.argtypes = [_D, _D, ctypes.c_double, _D, ctypes.POINTER(ctypes.c_int64)]
        L.orc_flux_limiter_box.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64), _D]
        L.orc_centre_limiter.argtypes = [_D, _D, ctypes.c_double, _D, ctypes.POINTER(ctypes.c_int64)]
        L.orc_vertex_root.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.orc_vertex_root.restype = ctypes.c_double
        L.orc_point_llf.argtypes = [_D, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _D]
        L.orc_simpson.argtypes = [ctypes.POINTER(_Params), _DD, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
        L.orc_cell_limiter.argtypes = [_D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _D, _D, _D, ctypes.POINTER(ctypes.c_int64)]
        L.orc_cell_diagnostics.argtypes = [ctypes.POINTER(_Params), _DD, _D, _D, _D]
        L.orc_divb.argtypes = [ctypes.POINTER(_Params), _DD, _D]
        _lib = L
    return _lib


def _params(prob, nthreads: int = 0) -> _Params:
    return _Params(int(prob.nx), int(prob.ny), float(prob.x0), float(prob.x1), float(prob.y0), float(prob.y1),
                   float(prob.gamma), float(prob.cfl), float(prob.kappa), int(prob.bc_x), int(prob.bc_y),
                   int(nthreads))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _ptrs(state):
    return (_D * 4)(*[_ptr(a) for a in state])


def empty_like_state(state):
    return tuple(np.empty_like(a) for a in state)


def copy_state(state):
    return tuple(np.ascontiguousarray(a, dtype=np.float64).copy() for a in state)


def stage(prob, k: int, un, uk, dt: float, counters: Counters | None = None, nthreads: int = 0):
    """Return a_k U^n + b_k FE(U^(k), dt) (one SSP-RK3 stage)."""
    out = empty_like_state(un)
    c = _Counters(0, 0, 0, 0, 0, 0, 0, 0, 0, 1.0)
    rc = lib().orc_stage(ctypes.byref(_params(prob, nthreads)), k, _ptrs(un), _ptrs(uk), _ptrs(out), dt,
                         ctypes.byref(c))
    if rc != 0:
        raise ValueError("oracle stage rejected its arguments (rc=%d)" % rc)
    if counters is not None:
        counters.add(c)
    return out


def dt(prob, u, t_remaining: float = float("inf"), nthreads: int = 0) -> float:
    return lib().orc_dt(ctypes.byref(_params(prob, nthreads)), _ptrs(u), t_remaining)


def step(prob, u, t_remaining: float = float("inf"), fixed_dt: float | None = None,
         counters: Counters | None = None, nthreads: int = 0):
    """One SSP-RK3 step; returns (new_state, dt)."""
    v = copy_state(u)
    d = ctypes.c_double(fixed_dt if fixed_dt is not None else 0.0)
    c = _Counters(0, 0, 0, 0, 0, 0, 0, 0, 0, 1.0)
    rc = lib().orc_step(ctypes.byref(_params(prob, nthreads)), _ptrs(v), t_remaining,
                        1 if fixed_dt is not None else 0, ctypes.byref(d), ctypes.byref(c))
    if rc != 0:
        raise ValueError("oracle step rejected its arguments (rc=%d)" % rc)
    if counters is not None:
        counters.add(c)
    return v, d.value


def run(prob, u, t_final: float, max_steps: int | None = None, counters: Counters | None = None,
        nthreads: int = 0, dts: list | None = None):
    """Advance to t_final (or max_steps steps).  Returns (state, t, nsteps)."""
    t, n = 0.0, 0
    while t < t_final * (1 - 1e-14) and (max_steps is None or n < max_steps):
        u, d = step(prob, u, t_final - t, counters=counters, nthreads=nthreads)
        if dts is not None:
            dts.append(d)
        t += d
        n += 1
    return u, t, n


# ---- building blocks (for the pins)
def _vec(u) -> np.ndarray:
    a = np.ascontiguousarray(u, dtype=np.float64)
    assert a.shape == (8,)
    return a


def pressure(u, gamma):
    return lib().orc_pressure(_ptr(_vec(u)), gamma)


def flux(u, gamma, direction):
    out = np.zeros(8)
    lib().orc_flux(_ptr(_vec(u)), gamma, direction, _ptr(out))
    return out


def fast_speed(u, gamma, direction):
    return lib().orc_fast_speed(_ptr(_vec(u)), gamma, direction)


def spectral_radius(u, gamma, direction):
    return lib().orc_spectral_radius(_ptr(_vec(u)), gamma, direction)


def alpha_llf(u, ut, gamma, direction):
    return lib().orc_alpha_llf(_ptr(_vec(u)), _ptr(_vec(ut)), gamma, direction)


def llf_flux(u, ut, gamma, direction):
    out = np.zeros(8)
    lib().orc_llf_flux(_ptr(_vec(u)), _ptr(_vec(ut)), gamma, direction, _ptr(out))
    return out


def fvs_derivative(w, gamma, direction, h):
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert w.shape == (5, 8)
    R = np.zeros(8)
    dB = ctypes.c_double(0.0)
    lib().orc_fvs_derivative(_ptr(w), gamma, direction, h, _ptr(R), ctypes.byref(dB))
    return R, dB.value


def point_limiter(uh, ul, gamma):
    out = np.zeros(8)
    nf = ctypes.c_int64(0)
    lib().orc_point_limiter(_ptr(_vec(uh)), _ptr(_vec(ul)), gamma, _ptr(out), ctypes.byref(nf))
    return out, nf.value


def flux_limiter_box(a1, H, gamma, eps_rho, eps_p):
    """Step (2) of the flux limiter.  Returns (Lambda[4], info) with info's
    ``lambda_before_fallback`` the box before the round-off fallback."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    assert H.shape == (4, 8)
    lam = np.zeros(4)
    pre = np.zeros(4)
    nn, it, nf = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    lib().orc_flux_limiter_box(_ptr(_vec(a1)), _ptr(H), gamma, eps_rho, eps_p, _ptr(lam), ctypes.byref(nn),
                               ctypes.byref(it), ctypes.byref(nf), _ptr(pre))
    return lam, {"n_newton": nn.value, "iters_max": it.value, "n_fallback": nf.value,
                 "lambda_before_fallback": pre}


def centre_limiter(uc, a, gamma):
    """The centre value uc limited towards the cell average a; returns
    (limited state, n_fallback)."""
    out = np.zeros(8)
    nf = ctypes.c_int64(0)
    lib().orc_centre_limiter(_ptr(_vec(uc)), _ptr(_vec(a)), gamma, _ptr(out), ctypes.byref(nf))
    return out, nf.value


def vertex_root(a1, d, gamma, eps_p):
    it = ctypes.c_int(0)
    r = lib().orc_vertex_root(_ptr(_vec(a1)), _ptr(_vec(d)), gamma, eps_p, ctypes.byref(it))
    return r, it.value


def cell_diagnostics(prob, u):
    """(limited centre [8,ny,nx], 9-point source [8,ny,nx], sensor [4,ny,nx])."""
    ny, nx = int(prob.ny), int(prob.nx)
    centre = np.zeros((8, ny, nx))
    source = np.zeros((8, ny, nx))
    sensor = np.zeros((4, ny, nx))
    lib().orc_cell_diagnostics(ctypes.byref(_params(prob)), _ptrs(u), _ptr(centre), _ptr(source), _ptr(sensor))
    return centre, source, sensor


def divb(prob, u):
    """(div1, div2): the two discrete divergences of Section 4's
    Orszag-Tang example."""
    out = np.zeros(2)
    lib().orc_divb(ctypes.byref(_params(prob)), _ptrs(u), _ptr(out))
    return float(out[0]), float(out[1])


def point_llf(u, left, right, down, up, dt, dx, dy, gamma):
    out = np.zeros(8)
    lib().orc_point_llf(_ptr(_vec(u)), _ptr(_vec(left)), _ptr(_vec(right)), _ptr(_vec(down)), _ptr(_vec(up)), dt,
                        dx, dy, gamma, _ptr(out))
    return out


def simpson(prob, u, direction, k, j):
    out = np.zeros(8)
    lib().orc_simpson(ctypes.byref(_params(prob)), _ptrs(u), direction, k, j, _ptr(out))
    return out


def cell_limiter(A, Fs, Fl, S_s, S_llf, dt, dx, dy, gamma):
    """Flux limiter steps (1)-(2) for one cell.  Fs, Fl: (4, 8) in the order
    L, R, D, U.  Returns (theta_src, Lambda[4], A_lim1[8], n_fallback)."""
    F = np.ascontiguousarray(np.concatenate([np.asarray(Fs, float), np.asarray(Fl, float)]), dtype=np.float64)
    assert F.shape == (8, 8)
    S = np.ascontiguousarray(np.stack([np.asarray(S_s, float), np.asarray(S_llf, float)]), dtype=np.float64)
    th = ctypes.c_double(0.0)
    lam = np.zeros(4)
    a1 = np.zeros(8)
    nf = ctypes.c_int64(0)
    lib().orc_cell_limiter(_ptr(_vec(A)), _ptr(F), _ptr(S), dt, dx, dy, gamma, ctypes.byref(th), _ptr(lam),
                           _ptr(a1), ctypes.byref(nf))
    return th.value, lam, a1, nf.value


# ---- tangent oracle: directional derivatives of the discrete map
_tlib = None


def tlib():
    global _tlib
    if _tlib is None:
        if not os.path.exists(TLIB):
            build(force=False)
        L = ctypes.CDLL(TLIB)
        L.orc_t_nd.restype = ctypes.c_int
        L.orc_t_stage.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _DD, _DD, _DD, _DD, _DD, _DD,
                                  ctypes.c_double]
        L.orc_t_stage.restype = ctypes.c_int
        L.orc_t_run.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _D, _DD, _DD]
        L.orc_t_run.restype = ctypes.c_int
        I64 = ctypes.POINTER(ctypes.c_int64)
        L.orc_t_point_limiter.argtypes = [_D, _D, _D, _D, ctypes.c_double, _D, _D, I64]
        L.orc_t_cell_limiter.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         _D, _D, _D, _D, I64]
        assert L.orc_t_nd() == TANGENT_ND
        _tlib = L
    return _tlib


def _stack_dirs(dirs, lo, state):
    """Directions lo .. lo+TANGENT_ND-1 (zeros past the end) as 4 arrays
    [TANGENT_ND, *shape of the set]."""
    out = []
    for q, a in enumerate(state):
        t = np.zeros((TANGENT_ND,) + a.shape)
        for d in range(TANGENT_ND):
            if lo + d < len(dirs):
                t[d] = dirs[lo + d][q]
        out.append(np.ascontiguousarray(t))
    return out


def tangent_stage(prob, k: int, un, dun, uk, duk, dt: float, nthreads: int = 0):
    """a_k U^n + b_k FE(U^(k), dt) and its derivatives along the directions
    (dun[d], duk[d]) (each a state-shaped tuple).  Returns (out, [dout_d])."""
    assert len(dun) == len(duk)
    out = empty_like_state(un)
    vn, vk = copy_state(un), copy_state(uk)  # kept alive across the call
    douts = []
    for lo in range(0, max(len(dun), 1), TANGENT_ND):
        tn, tk = _stack_dirs(dun, lo, un), _stack_dirs(duk, lo, uk)
        to = [np.empty_like(a) for a in tn]
        rc = tlib().orc_t_stage(ctypes.byref(_params(prob, nthreads)), k, _ptrs(vn), _ptrs(tn),
                                _ptrs(vk), _ptrs(tk), _ptrs(out), _ptrs(to), dt)
        if rc != 0:
            raise ValueError("tangent stage rejected its arguments (rc=%d)" % rc)
        for d in range(TANGENT_ND):
            if lo + d < len(dun):
                douts.append(tuple(np.ascontiguousarray(t[d]) for t in to))
    return out, douts


def tangent_run(prob, u, du, dts, nthreads: int = 0):
    """len(dts) SSP-RK3 steps with the given step sizes, with the derivatives
    along the directions du[d].  Returns (state, [d state_d])."""
    dts = np.ascontiguousarray(dts, dtype=np.float64)
    douts = []
    v = None
    for lo in range(0, max(len(du), 1), TANGENT_ND):
        v = copy_state(u)
        t = _stack_dirs(du, lo, u)
        rc = tlib().orc_t_run(ctypes.byref(_params(prob, nthreads)), len(dts), _ptr(dts), _ptrs(v), _ptrs(t))
        if rc != 0:
            raise ValueError("tangent run rejected its arguments (rc=%d)" % rc)
        for d in range(TANGENT_ND):
            if lo + d < len(du):
                douts.append(tuple(np.ascontiguousarray(x[d]) for x in t))
    return v, douts


def tangent_point_limiter(uh, ul, gamma, duh, dul):
    """Point scaling limiter with derivatives along up to TANGENT_ND
    directions: duh, dul are (n, 8).  Returns (out[8], dout[n, 8], n_fallback)."""
    n = len(duh)
    assert n <= TANGENT_ND
    D1 = np.zeros((TANGENT_ND, 8)); D1[:n] = duh
    D2 = np.zeros((TANGENT_ND, 8)); D2[:n] = dul
    out, dout, nf = np.zeros(8), np.zeros((TANGENT_ND, 8)), ctypes.c_int64(0)
    tlib().orc_t_point_limiter(_ptr(_vec(uh)), _ptr(D1), _ptr(_vec(ul)), _ptr(D2), gamma, _ptr(out), _ptr(dout),
                               ctypes.byref(nf))
    return out, dout[:n], nf.value


def tangent_cell_limiter(x, dx_dirs, dt, dx, dy, gamma):
    """Flux limiter steps (1)-(2) of one cell with derivatives.  x[88] =
    A, FsL, FsR, FsD, FsU, FlL, FlR, FlD, FlU, S_s, S_llf (8 each);
    dx_dirs (n, 88).  Returns (theta_src, dtheta[n], Lambda[4], dLambda[n, 4], n_fallback)."""
    n = len(dx_dirs)
    assert n <= TANGENT_ND
    x = np.ascontiguousarray(x, dtype=np.float64)
    D = np.zeros((TANGENT_ND, 88)); D[:n] = dx_dirs
    th, lam = ctypes.c_double(0.0), np.zeros(4)
    dth, dlam, nf = np.zeros(TANGENT_ND), np.zeros((TANGENT_ND, 4)), ctypes.c_int64(0)
    tlib().orc_t_cell_limiter(_ptr(x), _ptr(D), dt, dx, dy, gamma, ctypes.byref(th), _ptr(dth), _ptr(lam),
                              _ptr(dlam), ctypes.byref(nf))
    return th.value, dth[:n], lam, dlam[:n], nf.value
