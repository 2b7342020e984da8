"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the FP64 oracle (every entry point, every boundary kind, free
surface, windowed point steps, acoustic_iso) and the library's host runtime
(parameter checks, workspace layout and tile plans for every tile variant,
boundary kind, model, batch grouping and checkpoint setting, and the
clean-up of a context whose set-up stops at its first device call), and the
tile plans themselves (an optimised build: it visits every cell of every
plan): every cell written exactly once per step, the interior free of layer
cells, the CPML frame free of z-layer cells.  Any
invalid access, leak or undefined behaviour fails the run.  The GPU kernels
are not instrumented (GPU sanitizers are not available on these machines);
the kernel object is linked as built."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-std=c99", *SAN, "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe,
          "-lm"])
    assert "ok" in _run([exe], env=ENV, timeout=600)


def test_host_runtime_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2007_06048_amd", "csrc")
    kobj = os.path.join(csrc, "mm_kernels.o")
    if not os.path.exists(kobj):
        _run(["make", "-C", csrc, "mm_kernels.o"], timeout=900)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if shutil.which("g++") is None or not os.path.isdir(os.path.join(rocm, "include", "hip")):
        pytest.fail("g++ and the ROCm headers are needed for the host build")
    exe = str(tmp_path / "host_asan")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{csrc}",
          os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), os.path.join(csrc, "mm_api.cpp"), kobj,
          "-o", exe, f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib"], timeout=600)
    assert "ok" in _run([exe], env=ENV, timeout=600)


def test_tile_plans_cover_every_cell_once(tmp_path):
    csrc = os.path.join(ROOT, "paper_2007_06048_amd", "csrc")
    kobj = os.path.join(csrc, "mm_kernels.o")
    if not os.path.exists(kobj):
        _run(["make", "-C", csrc, "mm_kernels.o"], timeout=900)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "tiles")
    _run(["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{csrc}",
          os.path.join(ROOT, "tests", "sanitize", "tiles_driver.cpp"), kobj, "-o", exe, f"-L{rocm}/lib", "-lamdhip64",
          f"-Wl,-rpath,{rocm}/lib"], timeout=600)
    assert "cases ok" in _run([exe], timeout=600)


def test_host_logic_under_sanitizers(tmp_path):
    """The watchdog's schedule and result decoding, the parameter check of
    watch_every, and the CPML memory width per model."""
    csrc = os.path.join(ROOT, "paper_2007_06048_amd", "csrc")
    kobj = os.path.join(csrc, "mm_kernels.o")
    if not os.path.exists(kobj):
        _run(["make", "-C", csrc, "mm_kernels.o"], timeout=900)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "logic")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{csrc}",
          os.path.join(ROOT, "tests", "sanitize", "host_logic_driver.cpp"), kobj, "-o", exe, f"-L{rocm}/lib",
          "-lamdhip64", f"-Wl,-rpath,{rocm}/lib"], timeout=600)
    assert "ok" in _run([exe], env=ENV, timeout=300)
