"""Summaries of rocprofv3 CSV output (``--output-format csv``) for the
library's kernels: per-kernel launch statistics from ``*_kernel_stats.csv``
and, from ``*_counter_collection.csv`` files, HBM traffic per launch scaled
against a plain copy kernel of known size.

  python -m paper_2506_04857_amd.rocprof_summary kernels STATS_CSV
  python -m paper_2506_04857_amd.rocprof_summary traffic \\
      --fetch FETCH_CSV --write WRITE_CSV --copy-fetch CSV --copy-write CSV --copy-bytes N
  python -m paper_2506_04857_amd.rocprof_summary sq --insts CSV --busy CSV [--cus 256 --xcc 8]

FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; the copy kernel reads
and writes N bytes per dispatch, so each counter's scale factor is
(N / 1024) / (its reading on the copy kernel).

sq: per-wave instruction counts (SQ_INSTS_* / SQ_WAVES, from the --insts
pass) and busy fractions as rocprof's VALUBusy, 100 * SQ_ACTIVE_INST_* /
CUs / (GRBM_GUI_ACTIVE / XCCs) (from the --busy pass), each the mean over
the kernel's dispatches.
"""
from __future__ import annotations

import argparse
import csv
import os
import sys
from collections import defaultdict


def _rows(path):
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            yield {k.strip().lower(): (v.strip() if isinstance(v, str) else v) for k, v in r.items() if k}


def _short(name: str) -> str:
    """Kernel name without return type, namespaces and arguments; template
    arguments are kept (k_points<double> and k_points<float> differ)."""
    n = name.replace("(anonymous namespace)::", "").strip()
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0].strip()


def kernel_stats(path):
    out = []
    for r in _rows(path):
        out.append((_short(r["name"]), int(r["calls"]), float(r["averagens"]) / 1e3, float(r["minns"]) / 1e3,
                    float(r["maxns"]) / 1e3, float(r["percentage"])))
    return out


def counter_per_dispatch(path, counter: str):
    """{short kernel name: mean over dispatches of the counter's value}."""
    per = defaultdict(float)
    kern = {}
    for r in _rows(path):
        if r.get("counter_name") != counter:
            continue
        d = r["dispatch_id"]
        per[d] += float(r["counter_value"])  # several rows per dispatch are summed
        kern[d] = _short(r["kernel_name"])
    agg = defaultdict(list)
    for d, v in per.items():
        agg[kern[d]].append(v)
    return {k: sum(v) / len(v) for k, v in agg.items()}


def _copy_value(table):
    keys = [k for k in table if "copy" in k.lower()]
    if not keys:
        raise SystemExit("no copy kernel in the calibration counters")
    return max(table[k] for k in keys)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernels")
    a.add_argument("stats_csv")
    b = sub.add_parser("traffic")
    for f in ("fetch", "write", "copy-fetch", "copy-write"):
        b.add_argument("--" + f, required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    c = sub.add_parser("sq")
    c.add_argument("--insts", required=True)
    c.add_argument("--busy", required=True)
    c.add_argument("--cus", type=int, default=256)
    c.add_argument("--xcc", type=int, default=8)
    args = ap.parse_args(argv)
    if args.cmd == "sq":
        get = lambda path, name: counter_per_dispatch(path, name)
        waves = get(args.insts, "SQ_WAVES")
        ins = {n: get(args.insts, "SQ_INSTS_" + n) for n in
               ("VALU", "VALU_FMA_F64", "VALU_ADD_F64", "VALU_MUL_F64", "VALU_TRANS_F64", "LDS", "SALU")}
        grbm = get(args.busy, "GRBM_GUI_ACTIVE")
        av = get(args.busy, "SQ_ACTIVE_INST_VALU")
        al = get(args.busy, "SQ_ACTIVE_INST_LDS")
        conf = get(args.busy, "SQ_LDS_BANK_CONFLICT")
        print(f"{'kernel':<20} {'waves':>6} {'VALU':>6} {'FMA64':>6} {'ADD64':>6} {'MUL64':>6} {'TRANS64':>7} "
              f"{'LDS':>5} {'SALU':>5} {'VALU%':>7} {'LDS%':>6} {'LDSconfl':>9}")
        for k in sorted(waves):
            if not (k.startswith("k_points") or k.startswith("k_cells")) or k not in grbm:
                continue
            w = waves[k]
            per = {n: ins[n].get(k, 0.0) / w for n in ins}
            cyc = args.cus * grbm[k] / args.xcc
            print(f"{k:<20} {w:>6.0f} {per['VALU']:>6.0f} {per['VALU_FMA_F64']:>6.0f} {per['VALU_ADD_F64']:>6.0f} "
                  f"{per['VALU_MUL_F64']:>6.0f} {per['VALU_TRANS_F64']:>7.0f} {per['LDS']:>5.0f} {per['SALU']:>5.0f} "
                  f"{100 * av.get(k, 0.0) / cyc:>6.1f}% {100 * al.get(k, 0.0) / cyc:>5.1f}% {conf.get(k, 0.0):>9.3g}")
        # machine-readable: VALU wave-instructions per launch (bench.py reads these)
        for k in sorted(waves):
            if k.startswith("k_points") or k.startswith("k_cells") or k.startswith("k_dt"):
                print(f"valu_insts_per_launch.{k}: {ins['VALU'].get(k, 0.0):.0f}")
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        from bench import source_hash
        print(f"source_sha256: {source_hash()}")
        return
    if args.cmd == "kernels":
        print(f"{'kernel':<34} {'calls':>6} {'avg us':>10} {'min us':>10} {'max us':>10} {'share %':>8}")
        for k in kernel_stats(args.stats_csv):
            print(f"{k[0][:34]:<34} {k[1]:>6d} {k[2]:>10.2f} {k[3]:>10.2f} {k[4]:>10.2f} {k[5]:>8.2f}")
        return
    fetch = counter_per_dispatch(args.fetch, "FETCH_SIZE")
    write = counter_per_dispatch(args.write, "WRITE_SIZE")
    cf = _copy_value(counter_per_dispatch(args.copy_fetch, "FETCH_SIZE"))
    cw = _copy_value(counter_per_dispatch(args.copy_write, "WRITE_SIZE"))
    sf = args.copy_bytes / 1024.0 / cf
    sw = args.copy_bytes / 1024.0 / cw
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from bench import source_hash
    print(f"copy_bytes: {args.copy_bytes:.0f}")
    print(f"copy_fetch_kib: {cf:.1f}")
    print(f"copy_write_kib: {cw:.1f}")
    print(f"fetch_scale: {sf:.4f}")
    print(f"write_scale: {sw:.4f}")
    for k in sorted(fetch):
        if k in write and not k.startswith("__amd") and "at::native" not in k:
            print(f"fetch_kib_per_dispatch.{k}: {fetch[k]:.1f}")
            print(f"write_kib_per_dispatch.{k}: {write[k]:.1f}")
            print(f"traffic_bytes_per_launch.{k}: {1024.0 * (fetch[k] * sf + write[k] * sw):.0f}")
    print(f"source_sha256: {source_hash()}")


if __name__ == "__main__":
    main()
