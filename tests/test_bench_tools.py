"""The measurement tooling of bench.py on synthetic rocprofv3 output (CPU only): the byte
counters scaled by the copy probe, the trace summary, and the one-GPU contract."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SELL = "void rafem::(anonymous namespace)::k_sell<float, 1, true>(rafem::(anonymous namespace)::RowArgs<float>)"
COPY = "__amd_rocclr_copyBuffer"


def _counter_csv(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_counter_summary_scales_by_the_copy_probe(tmp_path, capsys):
    mib = 1024
    # FETCH_SIZE reads half of what a copy moves, WRITE_SIZE all of it (as measured)
    fetch = [(COPY, 0.5 * mib * 1024)] * 3 + [(COPY, 7.0)] + [(SELL, 60000.0)] * 5 + [(SELL, 3.0)] * 2
    write = [(COPY, 1.0 * mib * 1024)] * 3 + [(SELL, 4000.0)] * 5 + [(SELL, 1.0)] * 2
    _counter_csv(str(tmp_path / "f" / "host"), "FETCH_SIZE", fetch)
    _counter_csv(str(tmp_path / "w" / "host"), "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    out.write_text(json.dumps({"k_sell<float, 1, true> | C2 tet161 | nnz=5": {
        "kernel": "k_sell<float, 1, true>", "workload": "C2 tet161", "nnz": 5,
        "bytes_per_launch": 1.0}}))
    bench.counters_summary(str(tmp_path / "f"), str(tmp_path / "w"), mib, "C1 hex101", 27270901,
                           out_path=str(out))
    data = json.loads(out.read_text())
    # another workload's entry is kept, this one's is keyed by kernel, workload and nnz
    assert data["k_sell<float, 1, true> | C2 tet161 | nnz=5"]["bytes_per_launch"] == 1.0
    e = data[bench.traffic_key("k_sell<float, 1, true>", "C1 hex101", 27270901)]
    assert abs(e["fetch_size_copy_factor"] - 0.5) < 1e-12
    assert abs(e["write_size_copy_factor"] - 1.0) < 1e-12
    assert e["fetch_size_launches"] == 5 and e["write_size_launches"] == 5  # early exits dropped
    assert abs(e["fetch_size_bytes"] - 60000.0 * 1024 / 0.5) < 1e-6
    assert abs(e["bytes_per_launch"] - (60000.0 * 1024 / 0.5 + 4000.0 * 1024)) < 1e-6
    assert e["kernels_sha"] == bench.kernel_hash()
    assert "HBM bytes per launch" in capsys.readouterr().out


def test_trace_summary_tables(tmp_path, capsys):
    d = tmp_path / "prof" / "host"
    d.mkdir(parents=True)
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "TotalDurationNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": SELL, "Calls": 60, "AverageNs": 20000, "MinNs": 1000,
                    "TotalDurationNs": 1200000, "Percentage": 100.0})
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Start_Timestamp", "End_Timestamp", "Kernel_Name"])
        w.writeheader()
        t = 0
        for i in range(60):
            w.writerow({"Start_Timestamp": t, "End_Timestamp": t + 20000, "Kernel_Name": SELL})
            t += 21000  # 1 us gaps
    bench.trace_summary(str(tmp_path / "prof"))
    text = capsys.readouterr().out
    assert "k_sell<float, 1, true>" in text and "20.00" in text
    assert "median=  1.00" in text  # the gaps
    assert "n=   60 (of 60)" in text


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_step_stats_interval():
    import bench
    s = bench.step_stats([0.010, 0.012, 0.011, 0.013])
    assert abs(s["median_ms"] - 11.5) < 1e-9 and abs(s["mean_ms"] - 11.5) < 1e-9
    # 3 sigma / sqrt(n), sigma the sample standard deviation (1.2910 ms)
    assert abs(s["ci997_halfwidth_ms"] - 3 * 1.2909944487358056 / 2) < 1e-9
    assert bench.step_stats([0.01])["ci997_halfwidth_ms"] is None


def test_predictor_modes_of_the_simulation_driver():
    """sim's phys.extrapolate per step: off, a new trajectory, continuing it, and no history
    kept for the first step from a problem's initial state (its V is not a solution)."""
    from paper_2409_13036_amd.sim import _extrapolate_mode
    assert _extrapolate_mode(False, True, False) == 0
    assert _extrapolate_mode(True, False, False) == 2
    assert _extrapolate_mode(True, True, False) == 1
    assert _extrapolate_mode(True, False, True) == 0
    assert _extrapolate_mode(True, True, True) == 0
