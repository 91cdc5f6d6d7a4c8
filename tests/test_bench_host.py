"""Host-side logic of the benchmark script (no GPU): the multi-GPU refusal and
the scaling of the rocprofv3 traffic counters."""
import csv
import json
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
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _write_counters(path, counter, rows):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for d, name, value in rows:
            # counters come per hardware instance: split each value in two rows
            for part in (0.25, 0.75):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                            "Counter_Value": value * part})


def test_counter_scaling(tmp_path):
    gib = 1 << 30
    # a 1 GiB copy reads 524288 FETCH units (2048 B each) and writes 1048576
    # WRITE units (1024 B each); a small copy and two step launches besides
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    # two steps: ghost kernel, uniform-strip launch, mixed-strip launch each
    _write_counters(f, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 3.0),
                                      (2, "void pclb::ghost_kernel<float>", 7.0),
                                      (3, "void pclb::step_strip_kernel<2, false>", 1000.0),
                                      (4, "void pclb::step_strip_kernel<2, true>", 100.0),
                                      (5, "void pclb::ghost_kernel<float>", 7.0),
                                      (6, "void pclb::step_strip_kernel<2, false>", 2800.0),
                                      (7, "void pclb::step_strip_kernel<2, true>", 100.0),
                                      (8, "__amd_rocclr_copyBuffer", 524288.0)])
    _write_counters(w, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 1.0),
                                      (2, "void pclb::ghost_kernel<float>", 3.0),
                                      (3, "void pclb::step_strip_kernel<2, false>", 450.0),
                                      (4, "void pclb::step_strip_kernel<2, true>", 50.0),
                                      (5, "void pclb::ghost_kernel<float>", 3.0),
                                      (6, "void pclb::step_strip_kernel<2, false>", 1450.0),
                                      (7, "void pclb::step_strip_kernel<2, true>", 50.0),
                                      (8, "__amd_rocclr_copyBuffer", 1048576.0)])
    rec = bench.summarize_counters(str(f), str(w), nodes=1000)
    e = rec["fp32"]
    assert e["fetch_bytes"] == pytest.approx(2000.0 * gib / 524288.0)
    assert e["write_bytes"] == pytest.approx(1000.0 * gib / 1048576.0)
    assert e["bytes_per_launch"] == pytest.approx(e["fetch_bytes"] + e["write_bytes"])
    assert e["algorithmic_bytes"] == 2 * 33 * 1000 * 4
    assert rec["source_hash"] == bench.kernel_source_hash()
