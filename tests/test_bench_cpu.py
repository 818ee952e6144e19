"""Host-side parts of bench.py's contract, on the CPU: the one-GPU refusal,
and the HBM-traffic summary that scales rocprofv3's FETCH_SIZE / WRITE_SIZE
counters by what they read for the 1 GiB calibration copy."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write_counters(d, counter, rows):
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    with open(os.path.join(d, "host", "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path):
    gib_kib = (1 << 30) / 1024
    copy = "__amd_rocclr_copyBuffer"
    dot = "void pct::k_plan_dot<0, false>(pct::PlanView, long, float const*)"
    # the copy reads 1 GiB and writes 1 GiB; the counters see half the reads
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE",
                    [(copy, 10.0), (copy, 0.5 * gib_kib), (dot, 1000.0), (dot, 3000.0), ("at::other", 5.0)])
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", [(copy, 10.0), (copy, gib_kib), (dot, 400.0), (dot, 600.0)])
    out = str(tmp_path / "t.json")
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), out)
    t = json.load(open(out))
    assert abs(t["fetch_scale"] - 0.5) < 1e-12 and abs(t["write_scale"] - 1.0) < 1e-12
    assert t["source_hash"] == bench.source_hash()
    k = t["kernels"]["pct::k_plan_dot<0, false>"]
    assert k["dispatches"] == 2
    assert k["fetch_kib_per_dispatch"] == 2000.0 and k["write_kib_per_dispatch"] == 500.0
    assert "at::other" not in t["kernels"]
