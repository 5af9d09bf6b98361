"""Host logic of the benchmark (no GPU): the one-GPU refusal, and the
profile summaries it reads (copy-calibrated HBM traffic, gated on the hash
of the kernel source the counters were taken on)."""

import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2505_02350_amd import prof_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in msg["error"]


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_traffic_summary_is_copy_calibrated_and_hash_gated(tmp_path):
    fwd = "void erbf::k_forward<true, 256>(erbf::Dev, float*, float, float, int)"
    copy_bytes = 1 << 20   # 1024 KiB copied
    # the copy reads 2048 KiB and writes 512 KiB by the counters: scales 1/2 and 2
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(PS.COPY_KERNEL, 16.0), (PS.COPY_KERNEL, 2048.0), (fwd, 100.0), (fwd, 300.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(PS.COPY_KERNEL, 4.0), (PS.COPY_KERNEL, 512.0), (fwd, 10.0), (fwd, 30.0)])
    text = PS.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), copy_bytes, ["k_forward"],
                              "rocprofv3 --pmc FETCH_SIZE ...", "rocprofv3 --pmc WRITE_SIZE ...")
    out = tmp_path / "traffic.md"
    out.write_text(text)
    block = PS.read_traffic(str(out))
    assert block is not None
    assert block["scale_fetch"] == pytest.approx(0.5) and block["scale_write"] == pytest.approx(2.0)
    e = block["kernels"]["k_forward"]
    assert e["dispatches"] == 2
    # (200 KiB * 1/2 + 20 KiB * 2) per launch
    assert e["traffic_bytes_per_launch"] == pytest.approx(1024.0 * (100.0 + 40.0))
    # numbers taken on another kernel source are not used
    out.write_text(text.replace(block["source_sha256"], "0" * 64))
    assert PS.read_traffic(str(out)) is None
    assert PS.read_traffic(str(tmp_path / "missing.md")) is None


def test_traffic_summary_needs_the_calibration_copy(tmp_path):
    fwd = "erbf::k_bwd_tiles<4>(erbf::Dev, float const*, int)"
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [(fwd, 1.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(fwd, 1.0)])
    with pytest.raises(SystemExit):
        PS.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1024, ["k_bwd_tiles"], "a", "b")


def test_stats_table_rows(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "erbf::k_bwd_reduce(erbf::Dev, float const*, float*)", "Calls": 23,
                    "AverageNs": 21500.0, "MinNs": 20000.0, "MaxNs": 23700.0, "Percentage": 2.93})
    t = PS.stats_table(str(p), "title", "rocprofv3 --kernel-trace --stats -- python3 bench.py")
    assert "| `erbf::k_bwd_reduce(erbf::Dev, float const*, float*)` | 23 | 21.5 | 20.0 | 23.7 | 2.93 |" in t
