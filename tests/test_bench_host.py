"""Host-side checks of the measurement code in bench.py (no GPU): the algorithmic bytes each
roofline entry divides by, the choice of finest-level dispatches in counter summaries, the
scaling of FETCH_SIZE / WRITE_SIZE by the copy calibration, the idle fraction of a kernel trace,
and the refusal of more than one GPU."""
import csv
import importlib.util
import os
import sqlite3
import subprocess
import sys

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes_of_the_metric_workload(B):
    p = W.config3(0)
    nodes, N = 1025 ** 2, 512
    ab = B.algorithmic_bytes(p, 8)                         # FP32 slots: 8 bytes per complex value
    assert ab["residual_sweep"] == nodes * N * 8 + nodes * (N // 2) * 8
    assert ab["inverse_rfft_update"] == nodes * (N // 2) * 8 + 2 * nodes * N * 8
    assert ab["matvec_dot"] == nodes * (N // 2) * 8
    assert ab["vcycle_up_fine"] == 2 * nodes * (N // 2) * 8 + 513 ** 2 * (N // 2) * 8
    assert ab["vcycle_down_fine"] == nodes * (N // 2) * 8 + 513 ** 2 * (N // 2) * 8
    assert abs(ab["residual_sweep"] / 1e9 - 6.455) < 1e-3 and abs(ab["inverse_rfft_update"] / 1e9 - 10.758) < 1e-3
    # FP64 slots and a batch of four instances scale the slot and time-field terms
    ab64 = B.algorithmic_bytes(p, 16, count=4)
    assert ab64["matvec_dot"] == 4 * nodes * (N // 2) * 16


def _pmc_db(path, rows):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (dispatch_id int, kernel_name text, counter_name text, "
               "value real, duration real)")
    db.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    db.commit()
    db.close()


def test_counter_summary_takes_the_finest_level_and_scales_by_the_copy(B, tmp_path):
    # two levels of the up sweep (the coarse one short) and one residual sweep per step
    fetch = [(1, "void pt::k_vc_up<float, true, false, false>(...)", "FETCH_SIZE", 1000.0, 900.0),
             (2, "void pt::k_vc_up<float, true, false, false>(...)", "FETCH_SIZE", 250.0, 200.0),
             (3, "void pt::k_vc_up<float, true, false, false>(...)", "FETCH_SIZE", 1100.0, 950.0),
             (4, "void pt::k_residual<float, true, 1, 0, true, 0>(...)", "FETCH_SIZE", 3000.0, 1700.0)]
    write = [(r[0], r[1], "WRITE_SIZE", r[3] / 2, r[4]) for r in fetch]
    _pmc_db(tmp_path / "f.db", fetch)
    _pmc_db(tmp_path / "w.db", write)
    # the 1 GiB calibration copy reads as 512 MiB fetched and 1 GiB written
    _pmc_db(tmp_path / "cf.db", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 2.0 ** 19, 1.0)])
    _pmc_db(tmp_path / "cw.db", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 2.0 ** 20, 1.0)])
    out = tmp_path / "pmc.json"
    B.pmc_summary(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(tmp_path / "cf.db"), str(tmp_path / "cw.db"),
                  "c3", "fp32", str(out), "synthetic")
    import json
    data = json.loads(out.read_text())
    k = data["kernels"]["fp32"]
    assert data["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert data["calibration"]["write_factor"] == pytest.approx(1.0)
    # finest level only: dispatches 1 and 3 (at least half the longest), not the 250 KiB coarse one
    assert k["vcycle_up_fine"]["fetch_kib"] == pytest.approx(1050.0)
    assert k["vcycle_up_fine"]["read_bytes"] == pytest.approx(1050.0 * 1024 * 2)
    assert k["vcycle_up_fine"]["write_bytes"] == pytest.approx(525.0 * 1024)
    assert k["residual_sweep"]["hbm_bytes_per_launch"] == pytest.approx(3000.0 * 1024 * 2 + 1500.0 * 1024)


def test_trace_idle_fraction(B, tmp_path):
    # a warmup burst, an idle gap of 1 s, then kernels covering 9 of the window's 10 ms
    rows = [(0, 1_000_000, "warm"), (1_001_000_000, 1_005_000_000, "a"), (1_004_000_000, 1_006_000_000, "b"),
            (1_007_000_000, 1_011_000_000, "c")]
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Start_Timestamp", "End_Timestamp", "Kernel_Name"])
        w.writerows(rows)
    r = B.trace_idle(str(path))
    assert r["kernels_in_window"] == 3
    assert r["window_ms"] == pytest.approx(10.0)
    assert r["busy_ms"] == pytest.approx(9.0)
    assert r["idle_frac"] == pytest.approx(0.1)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
