"""ctypes driver of the host build of the adjoint's entity functions (test
infrastructure; see adjoint_hostcheck.cpp).  Built on demand with g++ into
tests/hostcheck/_build."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "adjoint_hostcheck.cpp")
CSRC = os.path.join(ROOT, "paper_2506_04857_amd", "csrc")
DEPS = [SRC, os.path.join(CSRC, "af_adjoint.h"), os.path.join(CSRC, "af_adjoint_stage.h")]
LIB = os.path.join(HERE, "_build", "libadjoint_hostcheck.so")

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_DD = ctypes.POINTER(_D)


class _P(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("gamma", ctypes.c_double),
                ("kappa", ctypes.c_double)]


def build() -> str:
    if os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-I", CSRC, SRC,
                           "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.hc_tape_bytes.argtypes = [ctypes.POINTER(_P)]
        L.hc_tape_bytes.restype = ctypes.c_size_t
        L.hc_adjbuf_bytes.argtypes = [ctypes.POINTER(_P)]
        L.hc_adjbuf_bytes.restype = ctypes.c_size_t
        L.hc_record.argtypes = [ctypes.POINTER(_P), ctypes.c_int, _DD, _DD, _DD, ctypes.c_double, ctypes.c_void_p]
        L.hc_adjoint.argtypes = [ctypes.POINTER(_P), ctypes.c_int, _DD, ctypes.c_void_p, ctypes.c_double, _DD, _DD,
                                 _DD, ctypes.c_void_p]
        U32, U64 = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
        dbl = ctypes.c_double
        L.hc_point_limit.argtypes = [_D, _D, dbl, _D, U32]
        L.hc_point_limit_vjp.argtypes = [_D, _D, dbl, ctypes.c_uint32, _D, _D, _D]
        L.hc_cell_limiter.argtypes = [_D, dbl, dbl, dbl, dbl, _D, _D, _D, U64]
        L.hc_cell_limiter_vjp.argtypes = [_D, dbl, dbl, dbl, dbl, _D, ctypes.c_uint64, dbl, _D, _D]
        _lib = L
    return _lib


def _params(prob):
    return _P(prob.nx, prob.ny, prob.bc_x, prob.bc_y, prob.dx, prob.dy, prob.gamma, prob.kappa)


def _ptrs(state):
    for a in state:
        assert a.dtype == np.float64 and a.flags.c_contiguous
    return (_D * 4)(*[a.ctypes.data_as(_D) for a in state])


def record(prob, k, un, uk, dt):
    """(stage output, tape bytes) of the recording forward."""
    p = _params(prob)
    tape = np.zeros(lib().hc_tape_bytes(ctypes.byref(p)) // 8 + 32)
    t = tape[(-tape.ctypes.data % 256) // 8:]
    out = tuple(np.zeros_like(a) for a in uk)
    lib().hc_record(ctypes.byref(p), k, _ptrs(un), _ptrs(uk), _ptrs(out), dt, t.ctypes.data_as(ctypes.c_void_p))
    return out, t


def adjoint(prob, k, uk, tape, dt, lam_out, lam_n=None, lam_k=None):
    """Accumulate lam_n += a_k lam_out, lam_k += b_k J^T lam_out (fresh zero
    accumulators when None); returns (lam_n, lam_k)."""
    p = _params(prob)
    lam_k = tuple(np.zeros_like(a) for a in uk) if lam_k is None else lam_k
    lam_n = (lam_k if k == 0 else tuple(np.zeros_like(a) for a in uk)) if lam_n is None else lam_n
    buf = np.zeros(lib().hc_adjbuf_bytes(ctypes.byref(p)) // 8 + 32)
    b = buf[(-buf.ctypes.data % 256) // 8:]
    lib().hc_adjoint(ctypes.byref(p), k, _ptrs(uk), tape.ctypes.data_as(ctypes.c_void_p), dt, _ptrs(lam_out),
                     _ptrs(lam_n), _ptrs(lam_k), b.ctypes.data_as(ctypes.c_void_p))
    return lam_n, lam_k


def _p(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def point_limit(uh, ul, gamma):
    """(out[8], decision bits)."""
    (uh, puh), (ul, pul) = _p(uh), _p(ul)
    out = np.zeros(8)
    fl = ctypes.c_uint32(0)
    lib().hc_point_limit(puh, pul, gamma, out.ctypes.data_as(_D), ctypes.byref(fl))
    return out, fl.value


def point_limit_vjp(uh, ul, gamma, fl, lout):
    (uh, puh), (ul, pul), (lo, plo) = _p(uh), _p(ul), _p(lout)
    a, b = np.zeros(8), np.zeros(8)
    lib().hc_point_limit_vjp(puh, pul, gamma, fl, plo, a.ctypes.data_as(_D), b.ctypes.data_as(_D))
    return a, b


def cell_limiter(x, dt, dx, dy, gamma):
    """(theta_src, Lambda[4], roots[15], decision bits) for x[88] = A, FsL..FsU,
    FlL..FlU, S_s, S_llf."""
    x, px = _p(x)
    th, lam, rk = ctypes.c_double(0.0), np.zeros(4), np.zeros(15)
    fl = ctypes.c_uint64(0)
    lib().hc_cell_limiter(px, dt, dx, dy, gamma, ctypes.byref(th), lam.ctypes.data_as(_D), rk.ctypes.data_as(_D),
                          ctypes.byref(fl))
    return th.value, lam, rk, fl.value


def cell_limiter_vjp(x, dt, dx, dy, gamma, rk, fl, lth, llam):
    (x, px), (rk, prk), (llam, pll) = _p(x), _p(rk), _p(llam)
    out = np.zeros(88)
    lib().hc_cell_limiter_vjp(px, dt, dx, dy, gamma, prk, fl, lth, pll, out.ctypes.data_as(_D))
    return out
