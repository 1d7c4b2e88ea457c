"""The measurement tooling on synthetic rocprofv3 CSV files (no GPU): the
per-dispatch counter means, the copy-calibrated traffic per launch, the SQ
summary, the bench's algorithmic byte counts and the committed summaries'
commands."""
import csv
import io
import os
import sys
from contextlib import redirect_stdout

import pytest

from paper_2506_04857_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
        "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
        "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_counters(path, rows):
    """rows: (dispatch, kernel name, counter, value); several rows of one
    dispatch and counter are summed by the reader (per-XCC rows)."""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEAD)
        for d, k, c, v in rows:
            w.writerow([d, d, "Agent 1", 1, 1, 1, 256, 1, k, 256, 0, 0, 8, 0, 16, c, v, 0, 1])


def run(argv):
    out = io.StringIO()
    with redirect_stdout(out):
        rs.main(argv)
    return out.getvalue()


def test_counter_means_sum_rows_of_a_dispatch(tmp_path):
    p = tmp_path / "c.csv"
    k = "void (anonymous namespace)::k_cells<double>(afm::Geo, afm::CState)"
    write_counters(p, [(1, k, "FETCH_SIZE", 10.0), (1, k, "FETCH_SIZE", 30.0), (2, k, "FETCH_SIZE", 60.0),
                       (2, k, "WRITE_SIZE", 5.0)])
    m = rs.counter_per_dispatch(str(p), "FETCH_SIZE")
    assert m == {"k_cells<double>": pytest.approx(50.0)}  # (40 + 60) / 2 dispatches


def test_traffic_scaled_by_the_copy_calibration(tmp_path):
    k = "void (anonymous namespace)::k_points<double>(afm::Geo)"
    copy = "void (anonymous namespace)::k_stream_copy(double2 const*, double2*, long)"
    write_counters(tmp_path / "f.csv", [(1, k, "FETCH_SIZE", 100.0)])
    write_counters(tmp_path / "w.csv", [(1, k, "WRITE_SIZE", 40.0)])
    # a copy of N bytes: FETCH_SIZE reads half of what it moves, WRITE_SIZE all of it
    n = 1024.0 * 1024.0
    write_counters(tmp_path / "cf.csv", [(1, copy, "FETCH_SIZE", n / 1024.0 / 2.0)])
    write_counters(tmp_path / "cw.csv", [(1, copy, "WRITE_SIZE", n / 1024.0)])
    txt = run(["traffic", "--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
               "--copy-fetch", str(tmp_path / "cf.csv"), "--copy-write", str(tmp_path / "cw.csv"),
               "--copy-bytes", str(n)])
    kv = dict(line.split(": ", 1) for line in txt.strip().splitlines())
    assert float(kv["fetch_scale"]) == pytest.approx(2.0)
    assert float(kv["write_scale"]) == pytest.approx(1.0)
    assert float(kv["traffic_bytes_per_launch.k_points<double>"]) == pytest.approx(1024.0 * (100.0 * 2.0 + 40.0))
    assert len(kv["source_sha256"]) == 64


def test_sq_summary_per_wave_counts_and_busy_fraction(tmp_path):
    k = "void (anonymous namespace)::k_points<double>(afm::Geo)"
    ins = [(1, k, "SQ_WAVES", 100.0), (1, k, "SQ_INSTS_VALU", 300000.0), (1, k, "SQ_INSTS_LDS", 5000.0)]
    for c in ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64",
              "SQ_INSTS_SALU"):
        ins.append((1, k, c, 100.0))
    write_counters(tmp_path / "a.csv", ins)
    # 256 CUs, 8 XCCs: GRBM_GUI_ACTIVE summed over XCCs = 8 * 1000 cycles
    write_counters(tmp_path / "b.csv", [(1, k, "GRBM_GUI_ACTIVE", 8000.0), (1, k, "SQ_ACTIVE_INST_VALU", 128000.0),
                                        (1, k, "SQ_ACTIVE_INST_LDS", 25600.0), (1, k, "SQ_LDS_BANK_CONFLICT", 0.0)])
    txt = run(["sq", "--insts", str(tmp_path / "a.csv"), "--busy", str(tmp_path / "b.csv")])
    row = [ln for ln in txt.splitlines() if ln.startswith("k_points<double>")][0].split()
    assert row[1] == "100" and row[2] == "3000"  # waves, VALU per wave
    assert row[9] == "50.0%" and row[10] == "10.0%"  # 128000 / 256 / 1000, 25600 / 256 / 1000
    kv = dict(ln.split(": ", 1) for ln in txt.splitlines() if ": " in ln)
    assert float(kv["valu_insts_per_launch.k_points<double>"]) == 300000.0  # what bench.py reads
    assert len(kv["source_sha256"]) == 64


def test_bench_algorithmic_bytes_per_cell():
    # k_points: read U^(k) 256 B, read X^n Y^n V^n 192 B (stages 1, 2), write
    # X Y V 192 B; k_cells: read U^(k) 256 B, read A^n 64 B (stages 1, 2),
    # write A 64 B; the stage: read U^(k) 256, U^n 256 (stages 1, 2), write
    # 256; means over the three stages
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    assert bench.BYTES_PER_CELL_POINTS == pytest.approx(256 + 192 + 192 * 2 / 3)
    assert bench.BYTES_PER_CELL_CELLS == pytest.approx(256 + 64 + 64 * 2 / 3)
    assert bench.BYTES_PER_CELL_STAGE == pytest.approx(256 + 256 + 256 * 2 / 3)


def test_bench_averages_the_last_stage_instantiation_over_a_step():
    # stages 0 and 1 run `<double, false>`, the last stage `<double, true>`
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    kv = {"traffic_bytes_per_launch.k_points<double, false>": "600",
          "traffic_bytes_per_launch.k_points<double, true>": "900",
          "traffic_bytes_per_launch.k_dt_from_parts": "70"}
    assert bench.stage_mean(kv, "traffic_bytes_per_launch", "k_points<double>") == pytest.approx(700.0)
    assert bench.stage_mean(kv, "traffic_bytes_per_launch", "k_dt_from_parts") == pytest.approx(70.0)
    assert bench.stage_mean(kv, "traffic_bytes_per_launch", "k_cells<double>") is None
    assert bench.stage_mean(None, "traffic_bytes_per_launch", "k_points<double>") is None


def test_bench_refuses_more_than_one_gpu():
    # the build runs on one GPU; bench.py --gpus N with N > 1 exits with a
    # message before touching any device
    import json
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_every_profile_summary_names_its_commands():
    # Each rocprofv3 summary under profiles/ is short text that gives the
    # full commands that made it (the profiler pass and the summariser), and
    # those commands run committed files only.
    import glob
    import re
    import subprocess
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))
    assert files
    # committed files: from git where the checkout has its history, else
    # the files present beside the tests
    res = subprocess.run(["git", "ls-files"], cwd=ROOT, capture_output=True, text=True)
    tracked = set(res.stdout.split()) if res.returncode == 0 else None
    for path in files:
        text = open(path).read()
        name = os.path.basename(path)
        assert len(text) < 16384, name
        assert "rocprofv3 " in text and "rocprof_summary" in text, name
        assert "_work" not in text, name
        for script in re.findall(r"\$R/(\S+\.py)\b", text):
            assert os.path.exists(os.path.join(ROOT, script)), (name, script)
            assert tracked is None or script in tracked, (name, script)
