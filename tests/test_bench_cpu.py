"""Host logic of bench.py (no GPU): the one-GPU refusal, the rocprofv3 CSV
summaries the committed profiles quote, and the HBM-traffic record."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def _write_csv(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_trace_summary_skips_and_takes_in_start_order(tmp_path, capsys):
    # dispatches listed out of start order: the summary sorts them by start
    rows = [
        {"Kernel_Name": "k_a", "Start_Timestamp": 300, "End_Timestamp": 330},   # 3rd: 30 ns
        {"Kernel_Name": "k_a", "Start_Timestamp": 100, "End_Timestamp": 190},   # 1st: 90 ns (warm-up)
        {"Kernel_Name": "k_a", "Start_Timestamp": 200, "End_Timestamp": 210},   # 2nd: 10 ns
        {"Kernel_Name": "k_a", "Start_Timestamp": 400, "End_Timestamp": 1400},  # 4th: 1000 ns
        {"Kernel_Name": "other", "Start_Timestamp": 50, "End_Timestamp": 60},
    ]
    sub = tmp_path / "run"
    sub.mkdir()
    _write_csv(sub / "run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    bench.trace_summary(str(tmp_path), 1, 2, "k_")
    out = capsys.readouterr().out.splitlines()
    body = [l for l in out if l.startswith("| `")]
    assert len(body) == 1                       # "other" does not match
    cells = [c.strip() for c in body[0].strip("|").split("|")]
    assert cells[0] == "`k_a`"
    assert cells[1:] == ["4", "1..2", "20", "10", "30"]   # dispatches 1 and 2: mean 20, min 10, max 30
    bench.trace_summary(str(tmp_path), 1, 0, "k_a")       # take 0: all after the skipped one
    cells = [c.strip() for c in [l for l in capsys.readouterr().out.splitlines()
                                 if l.startswith("| `")][0].strip("|").split("|")]
    assert cells[1:] == ["4", "1..3", "346", "10", "1000"]


def test_pmc_summary_averages_per_kernel_and_counter(tmp_path, capsys):
    rows = [
        {"Kernel_Name": "kern", "Counter_Name": "SQ_WAVES", "Counter_Value": 10},
        {"Kernel_Name": "kern", "Counter_Name": "SQ_WAVES", "Counter_Value": 30},
        {"Kernel_Name": "kern", "Counter_Name": "FETCH_SIZE", "Counter_Value": 5},
    ]
    _write_csv(tmp_path / "a_counter_collection.csv", ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    bench.pmc_summary(str(tmp_path))
    out = capsys.readouterr().out.splitlines()
    waves = [l for l in out if "SQ_WAVES" in l][0]
    fetch = [l for l in out if "FETCH_SIZE" in l][0]
    assert "dispatches=2" in waves and waves.endswith("avg=20")
    assert "dispatches=1" in fetch and fetch.endswith("avg=5")


def test_percentile_picks_ranked_elements():
    v = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert bench.percentile(v, 0) == 1.0
    assert bench.percentile(v, 50) == 3.0
    assert bench.percentile(v, 100) == 5.0
    assert bench.percentile([7.0], 90) == 7.0


def test_traffic_record_belongs_to_the_current_kernel():
    # The committed FETCH_SIZE / WRITE_SIZE record is tied to the int8
    # kernel's sources by hash; the bench reports traffic only while they match.
    t, how = bench.read_traffic()
    assert t is not None, how
    # calibrated bytes within a few percent of the window's algorithmic
    # traffic: 4-bit samples read once, int32 visibilities written once
    algorithmic = 512 * 4096 * 4096 + 4096 * (512 * 513 // 2) * 8
    assert 0.98 * algorithmic < t < 1.05 * algorithmic
    assert "copy-kernel calibration" in how
