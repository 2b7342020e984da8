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
    """With k_vcheck reading 2x and k_vdt2 writing 1x its true bytes, every
    step kernel's counters are scaled by 1/2 and 1, averaged per dispatch and
    summed over the kernels of a time step; other kernels are left out."""
    from paper_2007_06048_amd import workloads as W
    wl = W.smooth_240()
    n = wl.nx ** 3
    kib = 4.0 * n / 1024.0  # 4 N bytes in KiB
    step = "void mm::k_step<32, 2, 1, 0, 0, 256, false>(args)"
    trial = "void mm::k_step<64, 4, 1, 0, 0, 256, false>(args)"  # an autotuner trial: fewer dispatches
    cpml = "void mm::k_cstep<32, 1, 512, true, 0, false>(args)"
    other = "void mm::k_fill(args)"
    _counter_file(tmp_path / "f", "FETCH_SIZE", [("mm::k_vcheck(args)", 2 * kib), (step, 6 * kib), (step, 8 * kib),
                                                 (trial, 99 * kib), (cpml, 2 * kib), (cpml, 2 * kib),
                                                 (other, 50 * kib)])
    _counter_file(tmp_path / "w", "WRITE_SIZE", [("mm::k_vdt2(args)", kib), (step, kib), (step, kib), (trial, kib),
                                                 (cpml, 3 * kib), (cpml, 3 * kib), (other, 50 * kib)])
    out = tmp_path / "traffic.json"
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), "smooth240", str(out))
    e = json.load(open(out))[wl.name]
    assert set(e["kernels"]) == {step, cpml}
    assert e["kernels"][step]["dispatches"] == 2
    assert e["fetch_scale"] == pytest.approx(0.5) and e["write_scale"] == pytest.approx(1.0)
    assert e["kernels"][step]["fetch_bytes"] == pytest.approx(0.5 * 7 * 4 * n, rel=1e-9)
    assert e["kernels"][cpml]["write_bytes"] == pytest.approx(12 * n, rel=1e-9)
    assert e["fetch_bytes_per_step"] == pytest.approx((14 + 4) * n, rel=1e-9)
    assert e["write_bytes_per_step"] == pytest.approx((4 + 12) * n, rel=1e-9)
    assert e["bytes_per_step"] == e["fetch_bytes_per_step"] + e["write_bytes_per_step"]
    nb2 = 2 * wl.nb
    assert e["alg_bytes_per_step"] == 16 * n + 16 * 3 * nb2 * wl.nx * wl.nx
    assert e["kernel_hash"] == bench.kernel_hash()


def test_pmc_summary_keeps_kernel_durations_and_per_launch_fractions(tmp_path, monkeypatch):
    """With a --stats run beside the counters each kernel keeps its average
    duration; the bench line's per-launch breakdown then divides each part's
    algorithmic bytes by it (and is dropped once the kernel source changes)."""
    from types import SimpleNamespace as NS
    wl = NS(name="t", nx=128, ny=96, nz=80, bc=2, nb=8, free_surface=0)
    n = wl.nx * wl.ny * wl.nz
    kib = 4.0 * n / 1024.0
    names = {"interior": "void mm::k_step<64, 2, 1, 0, 0, 512, true, false>(a)",
             "frame": "void mm::k_cstep<32, 1, 512, 2, true, false, 0, true, false>(a)",
             "z_layer": "void mm::k_cstep<32, 1, 512, 2, false, true, 0, true, false>(a)",
             "z_corners": "void mm::k_cstep<32, 1, 512, 2, true, true, 0, true, false>(a)"}
    _counter_file(tmp_path / "f", "FETCH_SIZE", [("mm::k_vcheck(args)", kib)] + [(k, kib) for k in names.values()])
    _counter_file(tmp_path / "w", "WRITE_SIZE", [("mm::k_vdt2(args)", kib)] + [(k, kib) for k in names.values()])
    os.makedirs(tmp_path / "s")
    with open(tmp_path / "s" / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs"])
        w.writeheader()
        for i, k in enumerate(names.values()):
            w.writerow({"Name": k, "Calls": 20, "AverageNs": 1000.0 * (i + 1)})
    out = tmp_path / "traffic.json"
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), wl, str(out), str(tmp_path / "s"))
    e = json.load(open(out))["t"]
    assert e["kernels"][names["frame"]]["avg_ns"] == 2000.0 and e["kernels"][names["frame"]]["calls"] == 20
    monkeypatch.setattr(bench, "traffic_entry", lambda name: e)
    parts = bench.kernel_breakdown(wl)
    alg = bench.region_alg_bytes(wl)
    assert set(parts) == set(names)
    for i, kind in enumerate(names):
        assert parts[kind]["alg_bytes"] == alg[kind]
        assert parts[kind]["achieved"] == pytest.approx(alg[kind] / (1e-6 * (i + 1)) / 1e9, rel=1e-3)
        assert parts[kind]["traffic"] == round(4 * n) + round(4 * n)


def test_region_alg_bytes_sum_to_the_step():
    """The four parts of a fused CPML step (interior, frame, z-layer chunks,
    z-layer corners) add up to the whole step's algorithmic bytes."""
    from types import SimpleNamespace as NS
    for nx, ny, nz, nb in ((1024, 1024, 512, 32), (240, 240, 240, 20), (37, 29, 23, 5)):
        wl = NS(nx=nx, ny=ny, nz=nz, bc=2, nb=nb, free_surface=0)
        assert sum(bench.region_alg_bytes(wl).values()) == bench.step_alg_bytes(wl, 16)
    assert bench.launch_kind("void mm::k_cstep<32, 1, 512, 2, true, false, 0, true, false>(x)") == "frame"
    assert bench.launch_kind("void mm::k_cstep<32, 1, 512, 2, false, true, 1, false, true>(x)") == "z_layer"
    assert bench.launch_kind("void mm::k_cstep<32, 1, 512, 2, true, true, 0, false, false>(x)") == "z_corners"
    assert bench.launch_kind("void mm::k_step<64, 2, 1, 0, 0, 512, true, false>(x)") == "interior"


def test_step_alg_bytes_at_the_1024_workload():
    """20.0 bytes per point at 1024 x 1024 x 512 with a 32-cell CPML (16 B
    per point and 16 B per point and damped axis), 24.0 at 240^3 with 20."""
    from types import SimpleNamespace as NS
    a = bench.step_alg_bytes(NS(nx=1024, ny=1024, nz=512, bc=2, nb=32), 16)
    assert a / (1024 * 1024 * 512) == pytest.approx(20.0, abs=0.01)
    b = bench.step_alg_bytes(NS(nx=240, ny=240, nz=240, bc=2, nb=20), 16)
    assert b / 240 ** 3 == pytest.approx(24.0, abs=0.01)
    assert bench.step_alg_bytes(NS(nx=64, ny=64, nz=64, bc=1, nb=12), 16) == 16 * 64 ** 3
