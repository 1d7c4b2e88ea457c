"""The C-ABI library loads and exports every entry point that
include/af_mhd.h declares; host-side argument checks (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "af_mhd.h")
LIB = os.path.join(ROOT, "paper_2506_04857_amd", "libaf_mhd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(af_mhd_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libaf_mhd.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("af_mhd_init", "af_mhd_dt", "af_mhd_stage", "af_mhd_step", "af_mhd_workspace_bytes",
              "af_mhd_stats", "af_mhd_destroy", "af_mhd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_host_side_argument_checks(lib):
    from paper_2506_04857_amd import inputs as I
    from paper_2506_04857_amd.af_mhd import AF_EINVAL, af_mhd_params, make_params, load_library
    L = load_library(LIB)
    p = make_params(I.orszag_tang(64))
    n = L.af_mhd_workspace_bytes(ctypes.byref(p))
    # RK scratch (2 states x 256 B/cell) plus intermediates
    assert n > 2 * 8 * 32 * 64 * 64
    bad = make_params(I.orszag_tang(3))
    assert L.af_mhd_workspace_bytes(ctypes.byref(bad)) == 0
    h = ctypes.c_void_p()
    assert L.af_mhd_init(ctypes.byref(bad), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h)) == AF_EINVAL
    # misaligned workspace
    assert L.af_mhd_init(ctypes.byref(p), ctypes.c_void_p(8), 1 << 30, None, ctypes.byref(h)) == AF_EINVAL
    assert L.af_mhd_init(ctypes.byref(p), None, 1 << 30, None, ctypes.byref(h)) == AF_EINVAL
    assert L.af_mhd_stage(None, 0, None, None, None, None) == AF_EINVAL
    assert L.af_mhd_dt(None, None, 1.0, None) == AF_EINVAL
    assert L.af_mhd_step(None, None, 1.0, None) == AF_EINVAL
    from dataclasses import replace
    for q in (replace(I.orszag_tang(64), gamma=1.0), replace(I.orszag_tang(64), cfl=0.0),
              replace(I.orszag_tang(64), kappa=-1.0), replace(I.orszag_tang(64), bc_x=7)):
        assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(q))) == 0
    # flags: only the FP32-bulk, timing and fused-dt bits are accepted
    from paper_2506_04857_amd.af_mhd import AF_FLAG_FP32_BULK, AF_FLAG_FUSED_DT, AF_FLAG_KERNEL_TIMING
    assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(I.orszag_tang(64), AF_FLAG_KERNEL_TIMING))) == n
    assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(I.orszag_tang(64), AF_FLAG_FP32_BULK))) == n
    assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(I.orszag_tang(64), AF_FLAG_FUSED_DT))) == n
    assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(I.orszag_tang(64), 1 << 7))) == 0
    assert L.af_mhd_kernel_times(None, None, 0) == AF_EINVAL
    # the limiters entry: bad kind, flag or pointers are rejected on the host
    L.af_mhd_limiters_apply.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    assert L.af_mhd_limiters_apply(4, 1, 1.4, 256, 256, 0, 256, None) == AF_EINVAL
    assert L.af_mhd_limiters_apply(0, 1, 1.4, 256, 256, 2, 256, None) == AF_EINVAL
    assert L.af_mhd_limiters_apply(0, 1, 1.0, 256, 256, 0, 256, None) == AF_EINVAL
    assert L.af_mhd_limiters_apply(0, 1, 1.4, None, 256, 0, 256, None) == AF_EINVAL
    assert L.af_mhd_limiters_apply(0, -1, 1.4, 256, 256, 0, 256, None) == AF_EINVAL
    assert L.af_mhd_limiters_apply(0, 0, 1.4, None, None, 0, None, None) == 0


def test_batch_host_side_argument_checks(lib):
    from paper_2506_04857_amd import inputs as I
    from paper_2506_04857_amd.af_mhd import AF_EINVAL, AF_FLAG_FP32_BULK, af_mhd_params, make_params, load_library
    L = load_library(LIB)
    probs = [I.orszag_tang(64), I.alfven(32).with_size(40, 24), I.blast_lowbeta(16)]
    P = (af_mhd_params * 3)(*[make_params(p) for p in probs])
    n = L.af_mhd_batch_workspace_bytes(P, 3)
    # two scratch states and a centre buffer per instance at least
    need = sum(8 * 8 * (3 * p.nx * p.ny + (p.nxp * p.ny + p.nx * p.nyp + p.nxp * p.nyp) * 2) for p in probs)
    assert n >= need
    assert L.af_mhd_batch_workspace_bytes(P, 0) == 0
    mixed = (af_mhd_params * 2)(make_params(probs[0]), make_params(probs[1], AF_FLAG_FP32_BULK))
    assert L.af_mhd_batch_workspace_bytes(mixed, 2) == 0
    import ctypes
    h = ctypes.c_void_p()
    assert L.af_mhd_batch_init(P, 3, None, None, None, None, 0, None, None, ctypes.byref(h)) == AF_EINVAL
    assert L.af_mhd_batch_step(None, 1) == AF_EINVAL
    assert L.af_mhd_batch_set_launch_mode(None, 2) == AF_EINVAL
    mode = ctypes.c_int()
    assert L.af_mhd_batch_launch_mode(None, ctypes.byref(mode)) == AF_EINVAL
    assert b"bad argument" in L.af_mhd_batch_last_error(None)


def test_maximum_sizes(lib):
    # 65536 cells per direction is the largest grid accepted; the workspace
    # size is computed without overflow; one more is rejected.
    from dataclasses import replace
    from paper_2506_04857_amd import inputs as I
    from paper_2506_04857_amd.af_mhd import load_library, make_params
    L = load_library(LIB)
    big = replace(I.orszag_tang(64), nx=65536, ny=65536)
    n = L.af_mhd_workspace_bytes(ctypes.byref(make_params(big)))
    # two RK scratch states and a centre buffer: (2 * 4 + 1) * 8 planes of 65536^2 doubles at least
    assert n >= 9 * 8 * 8 * 65536 * 65536
    assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(replace(big, nx=65537)))) == 0
    assert L.af_mhd_workspace_bytes(ctypes.byref(make_params(replace(big, nx=4, ny=4)))) > 0


def test_bench_traffic_is_tied_to_the_kernel_sources():
    # bench.py reports the committed rocprofv3 traffic and VALU counts only
    # for the kernel sources they were measured on (their SHA-256 is stored
    # with them).
    import os
    import bench
    h = bench.source_hash()
    assert h == bench.source_hash() and len(h) == 64
    for wl, fname in bench.TRAFFIC_FILES.items():
        path = os.path.join(bench.PROFILES, fname)
        recorded = []
        if os.path.exists(path):
            with open(path) as fh:
                recorded = [ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("source_sha256")]
        t = bench.measured_traffic(wl, "k_points<double>")
        assert (t is not None) == (recorded == [h])
    assert bench.measured_traffic("alfven_32", "k_points<double>") is None
    assert bench.measured_valu("alfven_32", "k_points<double>") is None
