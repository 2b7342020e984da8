"""Host-side pieces of bench.py that need no GPU: the refusal of a multi-GPU
run, and the HBM-traffic summary built from rocprofv3 counter files (each
counter scaled by what it reads for kernels of known size)."""
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
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def _counter_file(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_pmc_summary_scales_by_the_calibration_kernels(tmp_path):
    """With k_vcheck reading 2x and k_vdt2 writing 1x its true bytes, the
    stencil's counters are scaled by 1/2 and 1, per dispatch."""
    from paper_2007_06048_amd import workloads as W
    n = W.smooth_240().nx ** 3
    kib = 4.0 * n / 1024.0  # 4 N bytes in KiB
    step = "void mm::k_step<32, 2, 1, 2, 0, 256, false>(args)"
    cpml = "void mm::k_cpml<false, false>(args)"
    _counter_file(tmp_path / "f", "FETCH_SIZE", [("mm::k_vcheck(args)", 2 * kib), (step, 6 * kib), (step, 8 * kib),
                                                 (cpml, 2 * kib)])
    _counter_file(tmp_path / "w", "WRITE_SIZE", [("mm::k_vdt2(args)", kib), (step, kib), (step, kib),
                                                 (cpml, 3 * kib)])
    out = tmp_path / "traffic.json"
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), "smooth240", str(out))
    e = json.load(open(out))["smooth_240^3_cpml20_1000steps"]
    assert e["dispatches"] == 2 and e["kernel"] == step
    assert e["fetch_scale"] == pytest.approx(0.5) and e["write_scale"] == pytest.approx(1.0)
    assert e["fetch_bytes_per_launch"] == pytest.approx(0.5 * 7 * 4 * n, rel=1e-9)
    assert e["write_bytes_per_launch"] == pytest.approx(4 * n, rel=1e-9)
    assert e["bytes_per_launch"] == e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    assert e["alg_bytes_per_launch"] == 16 * n
    assert e["cpml"][cpml]["fetch_bytes"] == pytest.approx(4 * n, rel=1e-9)
    assert e["cpml"][cpml]["write_bytes"] == pytest.approx(12 * n, rel=1e-9)
    assert e["kernel_hash"] == bench.kernel_hash()
