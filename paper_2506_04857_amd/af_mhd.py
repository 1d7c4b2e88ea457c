"""Thin Python binding of the HIP library (include/af_mhd.h): argument
marshalling only.  Every step of the stage runs in libaf_mhd.so; PyTorch
provides device memory and the stream.  There is no fallback path: if the
library is missing this module raises on import.

A state is a tuple ``(cell, xface, yface, vert)`` of contiguous float64 CUDA
(HIP) tensors with shapes ``(8, ny, nx)``, ``(8, ny, nxp)``, ``(8, nyp, nx)``,
``(8, nyp, nxp)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# AF_MHD_LIB selects another build of the same library (e.g. for A/B timing)
LIB_PATH = os.environ.get("AF_MHD_LIB") or os.path.join(_PKG, "libaf_mhd.so")

AF_OK, AF_EINVAL, AF_EHIP, AF_EWORKSPACE, AF_ENOTADMISSIBLE = 0, -1, -2, -3, -4
AF_BC_PERIODIC, AF_BC_OUTFLOW = 0, 1


class af_mhd_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("kappa", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("flags", ctypes.c_uint32),
    ]


class af_mhd_state(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_void_p), ("xface", ctypes.c_void_p), ("yface", ctypes.c_void_p),
                ("vert", ctypes.c_void_p)]


class af_mhd_stats_t(ctypes.Structure):
    _fields_ = [
        ("min_rho", ctypes.c_double), ("min_p", ctypes.c_double), ("mass", ctypes.c_double),
        ("min_theta", ctypes.c_double),
        ("n_llf_not_admissible", ctypes.c_int64), ("n_newton", ctypes.c_int64),
        ("newton_iters_max", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
        ("n_not_admissible", ctypes.c_int64), ("n_theta_active", ctypes.c_int64),
        ("n_point_limited", ctypes.c_int64), ("n_centre_limited", ctypes.c_int64),
        ("n_source_limited", ctypes.c_int64), ("n_dof_not_admissible", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


AF_FLAG_FP32_BULK = 1
AF_FLAG_KERNEL_TIMING = 4
AF_FLAG_FUSED_DT = 8
AF_BATCH_FLAT, AF_BATCH_PERSISTENT, AF_BATCH_FUSED = 0, 1, 2


class af_mhd_kernel_times_t(ctypes.Structure):
    _fields_ = [
        ("ms_points", ctypes.c_double), ("ms_cells", ctypes.c_double), ("ms_dt", ctypes.c_double),
        ("n_points", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("n_dt", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    # torch first: the process must hold one HIP runtime, and torch brings
    # its own copy of libamdhip64; loading the library first would bind it to
    # the system copy and make torch's streams and memory foreign to it.
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run __graft_entry__.build() "
                          "or python -m paper_2506_04857_amd.build")
    L = ctypes.CDLL(path)
    P, S, ST = ctypes.POINTER(af_mhd_params), ctypes.POINTER(af_mhd_state), ctypes.POINTER(af_mhd_stats_t)
    vp = ctypes.c_void_p
    L.af_mhd_workspace_bytes.argtypes = [P]
    L.af_mhd_workspace_bytes.restype = ctypes.c_size_t
    L.af_mhd_init.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.af_mhd_init.restype = ctypes.c_int
    L.af_mhd_dt.argtypes = [vp, S, ctypes.c_double, vp]
    L.af_mhd_dt.restype = ctypes.c_int
    L.af_mhd_stage.argtypes = [vp, ctypes.c_int, S, S, S, vp]
    L.af_mhd_stage.restype = ctypes.c_int
    L.af_mhd_step.argtypes = [vp, S, ctypes.c_double, vp]
    L.af_mhd_step.restype = ctypes.c_int
    L.af_mhd_stats.argtypes = [vp, S, ST]
    L.af_mhd_stats.restype = ctypes.c_int
    L.af_mhd_reset_counters.argtypes = [vp]
    L.af_mhd_reset_counters.restype = ctypes.c_int
    L.af_mhd_divb.argtypes = [vp, S, vp]
    L.af_mhd_divb.restype = ctypes.c_int
    L.af_mhd_kernel_times.argtypes = [vp, ctypes.POINTER(af_mhd_kernel_times_t), ctypes.c_int]
    L.af_mhd_kernel_times.restype = ctypes.c_int
    PA = ctypes.POINTER(af_mhd_params)
    L.af_mhd_batch_workspace_bytes.argtypes = [PA, ctypes.c_int]
    L.af_mhd_batch_workspace_bytes.restype = ctypes.c_size_t
    L.af_mhd_batch_init.argtypes = [PA, ctypes.c_int, S, vp, vp, vp, ctypes.c_size_t, vp, ctypes.c_char_p,
                                    ctypes.POINTER(vp)]
    L.af_mhd_batch_init.restype = ctypes.c_int
    L.af_mhd_batch_step.argtypes = [vp, ctypes.c_int]
    L.af_mhd_batch_step.restype = ctypes.c_int
    L.af_mhd_batch_tile.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.af_mhd_batch_tile.restype = ctypes.c_int
    L.af_mhd_batch_launch_mode.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.af_mhd_batch_launch_mode.restype = ctypes.c_int
    L.af_mhd_batch_set_launch_mode.argtypes = [vp, ctypes.c_int]
    L.af_mhd_batch_set_launch_mode.restype = ctypes.c_int
    L.af_mhd_batch_counters.argtypes = [vp, ST]
    L.af_mhd_batch_counters.restype = ctypes.c_int
    L.af_mhd_batch_destroy.argtypes = [vp]
    L.af_mhd_batch_destroy.restype = None
    L.af_mhd_batch_last_error.argtypes = [vp]
    L.af_mhd_batch_last_error.restype = ctypes.c_char_p
    L.af_mhd_destroy.argtypes = [vp]
    L.af_mhd_destroy.restype = None
    L.af_mhd_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.af_mhd_stream_copy.restype = ctypes.c_int
    L.af_mhd_limiters_apply.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, vp, vp, ctypes.c_uint32, vp, vp]
    L.af_mhd_limiters_apply.restype = ctypes.c_int
    L.af_mhd_step_noalloc.argtypes = [P, S, ctypes.c_double, vp, vp]
    L.af_mhd_step_noalloc.restype = ctypes.c_int
    L.af_mhd_adj_tape_bytes.argtypes = [P]
    L.af_mhd_adj_tape_bytes.restype = ctypes.c_size_t
    L.af_mhd_adj_workspace_bytes.argtypes = [P]
    L.af_mhd_adj_workspace_bytes.restype = ctypes.c_size_t
    L.af_mhd_adj_init.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.af_mhd_adj_init.restype = ctypes.c_int
    L.af_mhd_adj_record.argtypes = [vp, ctypes.c_int, S, S, S, vp, vp, ctypes.c_size_t]
    L.af_mhd_adj_record.restype = ctypes.c_int
    L.af_mhd_adj_stage.argtypes = [vp, ctypes.c_int, S, vp, ctypes.c_size_t, vp, S, S, S]
    L.af_mhd_adj_stage.restype = ctypes.c_int
    L.af_mhd_adj_destroy.argtypes = [vp]
    L.af_mhd_adj_destroy.restype = None
    L.af_mhd_adj_last_error.argtypes = [vp]
    L.af_mhd_adj_last_error.restype = ctypes.c_char_p
    L.af_mhd_last_error.argtypes = [vp]
    L.af_mhd_last_error.restype = ctypes.c_char_p
    return L


_lib = load_library()


class AfMhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"af_mhd error {code}: {msg}")
        self.code = code


def make_params(prob, flags: int = 0) -> af_mhd_params:
    """af_mhd_params from any object with nx, ny, x0, x1, y0, y1, gamma, cfl,
    kappa, bc_x, bc_y attributes."""
    return af_mhd_params(int(prob.nx), int(prob.ny), float(prob.x0), float(prob.x1), float(prob.y0),
                         float(prob.y1), float(prob.gamma), float(prob.cfl), float(prob.kappa), int(prob.bc_x),
                         int(prob.bc_y), int(flags))


def af_mhd_workspace_bytes(params: af_mhd_params) -> int:
    return int(_lib.af_mhd_workspace_bytes(ctypes.byref(params)))


def _state(u) -> af_mhd_state:
    for t in u:
        if t.dtype.itemsize != 8 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("state arrays must be contiguous float64 device tensors")
    return af_mhd_state(*[t.data_ptr() for t in u])


class Context:
    """Owns one af_mhd_ctx, its workspace and a device dt slot."""

    def __init__(self, prob, device=None, stream=None, flags: int = 0):
        import torch

        self.prob = prob
        self.params = make_params(prob, flags)
        nbytes = af_mhd_workspace_bytes(self.params)
        if nbytes == 0:
            raise AfMhdError(AF_EINVAL, "invalid parameters")
        self.device = torch.device(device if device is not None else "cuda")
        # one extra 256-byte block so the workspace base can be aligned
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.dt_dev = torch.zeros(1, dtype=torch.float64, device=self.device)
        h = ctypes.c_void_p()
        rc = _lib.af_mhd_init(ctypes.byref(self.params), ctypes.c_void_p(self._ws_ptr), nbytes,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != AF_OK:
            raise AfMhdError(rc, "af_mhd_init failed: " + _lib.af_mhd_last_error(None).decode())
        self._h = h

    def _check(self, rc: int, allow=(AF_OK,)):
        if rc not in allow:
            raise AfMhdError(rc, _lib.af_mhd_last_error(self._h).decode())
        return rc

    def af_mhd_dt(self, u, t_remaining: float = float("inf")):
        self._check(_lib.af_mhd_dt(self._h, ctypes.byref(_state(u)), t_remaining,
                                   ctypes.c_void_p(self.dt_dev.data_ptr())))
        return self.dt_dev

    def af_mhd_stage(self, k: int, un, uk, out, dt_dev=None):
        dt_dev = self.dt_dev if dt_dev is None else dt_dev
        self._check(_lib.af_mhd_stage(self._h, k, ctypes.byref(_state(un)), ctypes.byref(_state(uk)),
                                      ctypes.byref(_state(out)), ctypes.c_void_p(dt_dev.data_ptr())))
        return out

    def af_mhd_step(self, u, t_remaining: float = float("inf")):
        self._check(_lib.af_mhd_step(self._h, ctypes.byref(_state(u)), t_remaining,
                                     ctypes.c_void_p(self.dt_dev.data_ptr())))
        return u

    def af_mhd_stats(self, u) -> dict:
        st = af_mhd_stats_t()
        rc = _lib.af_mhd_stats(self._h, ctypes.byref(_state(u)), ctypes.byref(st))
        self._check(rc, allow=(AF_OK, AF_ENOTADMISSIBLE))
        d = st.as_dict()
        d["admissible"] = rc == AF_OK
        return d

    def af_mhd_reset_counters(self):
        self._check(_lib.af_mhd_reset_counters(self._h))

    def af_mhd_divb(self, u):
        """Device tensor (div1, div2) of the state u (enqueued)."""
        import torch
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        self._check(_lib.af_mhd_divb(self._h, ctypes.byref(_state(u)), ctypes.c_void_p(out.data_ptr())))
        return out

    def af_mhd_kernel_times(self, reset: bool = False) -> dict:
        kt = af_mhd_kernel_times_t()
        self._check(_lib.af_mhd_kernel_times(self._h, ctypes.byref(kt), int(bool(reset))))
        return kt.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _lib.af_mhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver(Context):
    """A context that also advances a state to a final time."""

    def run(self, u, t_final: float, max_steps: int = 10 ** 9, t0: float = 0.0):
        """SSP-RK3 steps on u (in place) until t_final, the last step
        shortened to land on it.  Reads each dt back (one synchronisation
        per step).  Returns (time reached, steps taken)."""
        t, n = float(t0), 0
        while t < t_final and n < max_steps:
            self.af_mhd_step(u, t_final - t)
            t += float(self.dt_dev.item())
            n += 1
        return t, n


class Batch:
    """Owns one af_mhd_batch: n independent grids stepped together in place.
    states: list of n device states (tuples of 4 tensors), kept alive here."""

    def __init__(self, probs, states, flags: int = 0, device=None, stream=None, tune_table=None,
                 t_remaining=None):
        import torch

        n = len(probs)
        self.probs = list(probs)
        self.states = list(states)
        self.params = (af_mhd_params * n)(*[make_params(p, flags) for p in probs])
        nbytes = int(_lib.af_mhd_batch_workspace_bytes(self.params, n))
        if nbytes == 0:
            raise AfMhdError(AF_EINVAL, "invalid batch parameters")
        self.device = torch.device(device if device is not None else "cuda")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) & ~255
        # a stream of its own by default: hipGraph capture needs a non-null stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.dt_dev = torch.zeros(n, dtype=torch.float64, device=self.device)
        self.t_rem = None
        if t_remaining is not None:
            self.t_rem = torch.as_tensor(t_remaining, dtype=torch.float64).to(self.device).contiguous()
        torch.cuda.synchronize(self.device)  # the states and tables are ready before the batch's stream runs
        self._st = (af_mhd_state * n)(*[_state(u) for u in self.states])
        h = ctypes.c_void_p()
        rc = _lib.af_mhd_batch_init(self.params, n, self._st, ctypes.c_void_p(self.dt_dev.data_ptr()),
                                    ctypes.c_void_p(self.t_rem.data_ptr() if self.t_rem is not None else None),
                                    ctypes.c_void_p(ws), nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                    tune_table.encode() if tune_table else None, ctypes.byref(h))
        if rc != AF_OK:
            raise AfMhdError(rc, "af_mhd_batch_init failed: " + _lib.af_mhd_batch_last_error(None).decode())
        self._h = h
        self.n = n

    def _check(self, rc: int):
        if rc != AF_OK:
            raise AfMhdError(rc, _lib.af_mhd_batch_last_error(self._h).decode())
        return rc

    def step(self, use_graph: bool = True):
        """One step of every instance, enqueued on self.stream (synchronise
        it before reading the states from another stream)."""
        self._check(_lib.af_mhd_batch_step(self._h, int(bool(use_graph))))

    def tile(self, m: int):
        tx, ty = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.af_mhd_batch_tile(self._h, m, ctypes.byref(tx), ctypes.byref(ty)))
        return tx.value, ty.value

    def launch_mode(self) -> int:
        """AF_BATCH_FLAT, AF_BATCH_PERSISTENT or AF_BATCH_FUSED."""
        p = ctypes.c_int()
        self._check(_lib.af_mhd_batch_launch_mode(self._h, ctypes.byref(p)))
        return p.value

    def set_launch_mode(self, mode: int):
        self._check(_lib.af_mhd_batch_set_launch_mode(self._h, int(mode)))

    def persistent(self) -> bool:
        """Whether the stages run on persistent workgroups."""
        return self.launch_mode() == AF_BATCH_PERSISTENT

    def counters(self) -> dict:
        st = af_mhd_stats_t()
        self._check(_lib.af_mhd_batch_counters(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _lib.af_mhd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adjoint:
    """Owns one af_mhd_adj (the recorded stage and its reverse sweep) and its
    workspace.  FP64 only."""

    def __init__(self, prob, device=None, stream=None):
        import torch

        self.prob = prob
        self.params = make_params(prob, 0)
        nbytes = int(_lib.af_mhd_adj_workspace_bytes(ctypes.byref(self.params)))
        if nbytes == 0:
            raise AfMhdError(AF_EINVAL, "invalid parameters")
        self.tape_bytes = int(_lib.af_mhd_adj_tape_bytes(ctypes.byref(self.params)))
        self.device = torch.device(device if device is not None else "cuda")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = _lib.af_mhd_adj_init(ctypes.byref(self.params), ctypes.c_void_p(ws), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != AF_OK:
            raise AfMhdError(rc, "af_mhd_adj_init failed: " + _lib.af_mhd_adj_last_error(None).decode())
        self._h = h

    def _check(self, rc: int):
        if rc != AF_OK:
            raise AfMhdError(rc, _lib.af_mhd_adj_last_error(self._h).decode())

    def new_tape(self):
        """A device buffer for one stage's tape (256-byte aligned view)."""
        import torch

        buf = torch.empty(self.tape_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        return buf[off:off + self.tape_bytes]

    def record(self, k: int, un, uk, out, dt_dev, tape):
        """out = a_k un + b_k FE(uk, dt) and the stage's tape."""
        self._check(_lib.af_mhd_adj_record(self._h, k, ctypes.byref(_state(un)), ctypes.byref(_state(uk)),
                                           ctypes.byref(_state(out)), ctypes.c_void_p(dt_dev.data_ptr()),
                                           ctypes.c_void_p(tape.data_ptr()), tape.numel()))
        return out

    def stage(self, k: int, uk, tape, dt_dev, lam_out, lam_n, lam_k):
        """lam_n += a_k lam_out; lam_k += b_k J^T lam_out (k = 0: lam_n unused)."""
        ln = ctypes.byref(_state(lam_n)) if lam_n is not None else None
        self._check(_lib.af_mhd_adj_stage(self._h, k, ctypes.byref(_state(uk)), ctypes.c_void_p(tape.data_ptr()),
                                          tape.numel(), ctypes.c_void_p(dt_dev.data_ptr()),
                                          ctypes.byref(_state(lam_out)), ln, ctypes.byref(_state(lam_k))))

    def close(self):
        if getattr(self, "_h", None):
            _lib.af_mhd_adj_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CheckpointedRun:
    """n SSP-RK3 steps of one grid with the gradient of their end state by
    the discrete adjoint and sqrt(n) checkpointing.

    forward(): the recording stage advances the state and the dt of every
    step stays in device memory.  When every step's stage inputs and tapes
    fit the memory budget (keep_tapes=None: half of the device memory free
    when forward() starts; True: always; False: never) the forward keeps
    them all and backward(lam) sweeps them in reverse order, so the
    decisions the backward freezes are the forward's own tapes.  Otherwise
    the forward keeps only the state every `every` steps (default
    ceil(sqrt(n))) and its tapes go to one reusable buffer; backward(lam)
    then recomputes each segment, last first, from its checkpoint with the
    recording stage (stage inputs and tapes, 3 per step) before sweeping
    it.  The recording stage is deterministic, so that recomputation takes
    exactly the forward's decisions and reproduces its states bit for bit:
    either way the gradient is that of the trajectory forward() returned.
    With record_forward=False the fast stage kernels advance the forward
    instead (equal to the recording stage only to rounding, so the decisions
    the backward freezes are those of a trajectory within rounding of the
    returned one; tapes are then never kept).  The dt sequence is data
    (frozen), not differentiated."""

    def __init__(self, prob, device=None, every: int | None = None, record_forward: bool = True,
                 keep_tapes: bool | None = None):
        import torch

        self.prob = prob
        self.device = torch.device(device if device is not None else "cuda")
        self.ctx = Context(prob, device=self.device)
        self.adj = Adjoint(prob, device=self.device, stream=self.ctx.stream)
        self.every = every
        self.record_forward = record_forward
        self.keep_tapes = keep_tapes
        self.kept = None  # per step (U^n, U^(1), U^(2), tape0, tape1, tape2, dt) when the tapes are kept
        self.tapes_kept = False
        self.dts = None
        self.checkpoints = []
        self.recomputed_end = None

    def _zeros(self):
        import torch

        return tuple(torch.zeros(s, dtype=torch.float64, device=self.device) for s in self.prob.shapes())

    def _empty(self):
        import torch

        return tuple(torch.empty(s, dtype=torch.float64, device=self.device) for s in self.prob.shapes())

    def _zero_states(self, n: int):
        """n zeroed states carved from one buffer (one fill launch)."""
        import math

        import torch

        shapes = self.prob.shapes()
        sizes = [math.prod(s) for s in shapes]
        buf = torch.zeros(n * sum(sizes), dtype=torch.float64, device=self.device)
        out, off = [], 0
        for _ in range(n):
            st = []
            for s, m in zip(shapes, sizes):
                st.append(buf[off:off + m].view(s))
                off += m
            out.append(tuple(st))
        return out

    def forward(self, u0, nsteps: int, dts=None, t_final: float = float("inf")):
        """Returns the end state (new tensors) after nsteps steps, or fewer
        when t_final is reached first (each step's dt is capped by the time
        remaining; self.nsteps holds the steps taken).  dts: a device tensor
        of fixed step sizes to use instead of the CFL rule."""
        import math

        import torch

        every = self.every or max(1, math.isqrt(max(nsteps - 1, 0)) + 1)
        self.every = every
        u = tuple(t.clone() for t in u0)
        self.nsteps = nsteps
        self.checkpoints = []
        self.kept = None
        if dts is not None:
            self.dts = dts.to(self.device, torch.float64).contiguous()
            assert self.dts.numel() >= nsteps
        else:
            self.dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=self.device)
        keep = self.record_forward and self._keep(nsteps)
        self.tapes_kept = keep
        if keep:
            self.kept = []
        s1 = s2 = s3 = tape = None
        if not keep:
            s1, s2 = self._zeros(), self._zeros()
            s3 = self._zeros() if self.record_forward else None
            tape = self.adj.new_tape() if self.record_forward else None
        t = 0.0
        for s in range(nsteps):
            if math.isfinite(t_final) and t >= t_final:
                self.nsteps = s  # t_final reached: the run ends here
                break
            if s % every == 0 and not keep:
                self.checkpoints.append(tuple(x.clone() for x in u))
            rem = t_final - t if math.isfinite(t_final) else float("inf")
            d = self.dts[s:s + 1]
            if self.record_forward:
                if dts is None:
                    self.ctx.af_mhd_dt(u, rem)
                    d.copy_(self.ctx.dt_dev)
                if keep:
                    # the recording stage writes every element of its output
                    s1, s2, s3 = self._empty(), self._empty(), self._empty()
                    t0, t1, t2 = self.adj.new_tape(), self.adj.new_tape(), self.adj.new_tape()
                    self.adj.record(0, u, u, s1, d, t0)
                    self.adj.record(1, u, s1, s2, d, t1)
                    self.adj.record(2, u, s2, s3, d, t2)
                    self.kept.append((u, s1, s2, t0, t1, t2, d))
                    u = s3
                else:
                    self.adj.record(0, u, u, s1, d, tape)
                    self.adj.record(1, u, s1, s2, d, tape)
                    self.adj.record(2, u, s2, s3, d, tape)
                    u, s3 = s3, u
            elif dts is None:
                self.ctx.af_mhd_step(u, rem)
                d.copy_(self.ctx.dt_dev)
            else:
                self.ctx.af_mhd_stage(0, u, u, s1, d)
                self.ctx.af_mhd_stage(1, u, s1, s2, d)
                self.ctx.af_mhd_stage(2, u, s2, u, d)
            if math.isfinite(t_final):
                t += float(d.item())  # the time reached (one synchronisation per step)
        if keep:
            return tuple(x.clone() for x in u)  # the caller's; the kept inputs are the run's
        return u

    def step_bytes(self) -> int:
        """Device bytes one kept step holds: three stage inputs and three tapes."""
        import math

        state = 8 * sum(math.prod(s) for s in self.prob.shapes())
        return 3 * state + 3 * (self.adj.tape_bytes + 256)

    def _keep(self, nsteps: int) -> bool:
        import torch

        if self.keep_tapes is not None:
            return bool(self.keep_tapes)
        free, _ = torch.cuda.mem_get_info(self.device)
        return nsteps * self.step_bytes() <= free // 2

    def backward(self, lam_T):
        """Adjoint of the initial state given lam_T, the adjoint of the end
        state (a tuple of 4 device tensors, not modified)."""
        lam = tuple(x.clone() for x in lam_T)
        if self.kept is not None:
            # the forward's own stage inputs and tapes, last step first; each
            # is released once swept
            while self.kept:
                un, u1, u2, t0, t1, t2, d = self.kept.pop()
                ln, l2, l1 = self._zero_states(3)
                self.adj.stage(2, u2, t2, d, lam, ln, l2)
                self.adj.stage(1, u1, t1, d, l2, ln, l1)
                self.adj.stage(0, un, t0, d, l1, None, ln)
                lam = ln
            self.kept = None
            return lam
        every = self.every
        for c in reversed(range(len(self.checkpoints))):
            first = c * every
            last = min(first + every, self.nsteps)
            hist = []
            u = self.checkpoints[c]
            for s in range(first, last):
                d = self.dts[s:s + 1]
                # the recording stage writes every element of its output
                u1, u2, u3 = self._empty(), self._empty(), self._empty()
                t0, t1, t2 = self.adj.new_tape(), self.adj.new_tape(), self.adj.new_tape()
                self.adj.record(0, u, u, u1, d, t0)
                self.adj.record(1, u, u1, u2, d, t1)
                self.adj.record(2, u, u2, u3, d, t2)
                hist.append((u, u1, u2, t0, t1, t2, d))
                u = u3
            if c == len(self.checkpoints) - 1:
                self.recomputed_end = u  # the recomputed end state (equal to forward's)
            for un, u1, u2, t0, t1, t2, d in reversed(hist):
                # the sweep adds into its accumulators
                ln, l2, l1 = self._zero_states(3)
                self.adj.stage(2, u2, t2, d, lam, ln, l2)
                self.adj.stage(1, u1, t1, d, l2, ln, l1)
                self.adj.stage(0, un, t0, d, l1, None, ln)
                lam = ln
            del hist
        return lam

    def close(self):
        self.kept = None
        self.checkpoints = []
        self.adj.close()
        self.ctx.close()


def evolve(prob, u0, nsteps: int, every: int | None = None, dts=None, keep_tapes: bool | None = None):
    """End state of nsteps SSP-RK3 steps from u0 (4 float64 device tensors)
    as a differentiable torch function: backward runs the discrete adjoint
    over the forward's kept tapes or with sqrt(n) checkpointing
    (CheckpointedRun; decisions of the limiters and the sensor frozen as the
    forward took them, dt sequence fixed)."""
    import torch

    class _Evolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, *u):
            run = CheckpointedRun(prob, device=u[0].device, every=every, keep_tapes=keep_tapes)
            out = run.forward(tuple(x.detach() for x in u), nsteps, dts=dts)
            ctx.run = run
            return out

        @staticmethod
        def backward(ctx, *g):
            run = ctx.run
            lam_T = tuple(gi.contiguous() if gi is not None else torch.zeros(s, dtype=torch.float64,
                                                                              device=run.device)
                          for gi, s in zip(g, prob.shapes()))
            lam0 = run.backward(lam_T)
            run.close()
            return lam0

    return _Evolve.apply(*u0)


def stream_copy(src, dst, stream=None):
    """dst <- src with the library's stream-copy kernel (contiguous float64
    device tensors of the same even length), enqueued on stream."""
    import torch

    if src.dtype != torch.float64 or dst.dtype != torch.float64 or src.numel() != dst.numel():
        raise ValueError("stream_copy: float64 tensors of equal size")
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    rc = _lib.af_mhd_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(),
                                 ctypes.c_void_p(s.cuda_stream))
    if rc != AF_OK:
        raise AfMhdError(rc, "af_mhd_stream_copy failed")


def af_mhd_step_noalloc(prob, u, dt_dev, t_remaining=float("inf"), flags=0, stream=None):
    """One SSP-RK3 step in place on the device state u through the
    entry point that allocates nothing (scratch in the library's static
    device array; grids up to about 256 x 256 cells).  Enqueued."""
    import torch

    p = make_params(prob, flags)
    s = stream if stream is not None else torch.cuda.current_stream(u[0].device)
    rc = _lib.af_mhd_step_noalloc(ctypes.byref(p), ctypes.byref(_state(u)), t_remaining,
                                  ctypes.c_void_p(dt_dev.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    if rc != AF_OK:
        raise AfMhdError(rc, _lib.af_mhd_last_error(None).decode())


AF_LIM_POINT, AF_LIM_CENTRE, AF_LIM_SOURCE, AF_LIM_BOX = 0, 1, 2, 3
AF_LIM_NO_SHORTCUT = 1
_LIM_WIDTHS = {AF_LIM_POINT: (16, 8), AF_LIM_CENTRE: (16, 8), AF_LIM_SOURCE: (25, 9), AF_LIM_BOX: (42, 4)}
COUNTER_NAMES = ("n_llf_not_admissible", "n_newton", "newton_iters_max", "n_fallback", "n_not_admissible",
                 "n_theta_active", "n_point_limited", "n_centre_limited", "n_source_limited", "min_theta_bits")


def af_mhd_limiters_apply(kind, inputs, gamma, flags=0, stream=None):
    """The stage's limiter of the given kind on each row of inputs (a
    float64 device tensor [n, width]); returns (outputs [n, width_out],
    counters dict).  Synchronises."""
    import torch

    w_in, w_out = _LIM_WIDTHS[kind]
    if inputs.dtype != torch.float64 or inputs.dim() != 2 or inputs.shape[1] != w_in or not inputs.is_contiguous():
        raise ValueError("limiters_apply: contiguous float64 [n, %d] device tensor" % w_in)
    out = torch.empty((inputs.shape[0], w_out), dtype=torch.float64, device=inputs.device)
    cnt = torch.zeros(len(COUNTER_NAMES), dtype=torch.int64, device=inputs.device)
    s = stream if stream is not None else torch.cuda.current_stream(inputs.device)
    rc = _lib.af_mhd_limiters_apply(kind, inputs.shape[0], gamma, ctypes.c_void_p(inputs.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), flags, ctypes.c_void_p(cnt.data_ptr()),
                                    ctypes.c_void_p(s.cuda_stream))
    if rc != AF_OK:
        raise AfMhdError(rc, "af_mhd_limiters_apply failed")
    s.synchronize()
    return out, dict(zip(COUNTER_NAMES, cnt.cpu().tolist()))


def to_device(state, device="cuda"):
    import torch

    return tuple(torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(device).contiguous()
                 for a in state)


def to_host(state):
    return tuple(t.detach().cpu().numpy() for t in state)


def empty_state(prob, device="cuda"):
    import torch

    return tuple(torch.empty(s, dtype=torch.float64, device=device) for s in prob.shapes())
