"""Host-side memory safety of the batched-solve bookkeeping (CPU only).

The library's host code (api.cpp, setup.cpp) is built with AddressSanitizer
and UndefinedBehaviorSanitizer against tests/host_asan/stub_hip.cpp, a
host-only stand-in for the HIP runtime (captured graphs run their recorded
operations when launched) and for the kernels.  The harness runs the batch
sizes of the GPU batch tests -- 16 solves on 65^2 / 129^2 grids and the
64-solve workload on 257^2 / 513^2 / 1025^2 grids with 4..16 channels and the
real host setup (bound states, channel factors, coarsest inverses) -- over
several restart rounds in which the solves finish at different rounds, then
each solve alone, then the batch with an iteration limit between the solves'
needs, and destroys everything.  Any invalid access, use after free or leak
fails the run.
"""
import os
import shutil
import subprocess

import pytest

from paper_1412_1953_amd.workloads import batch_workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "paper_1412_1953_amd", "csrc", f) for f in ("api.cpp", "setup.cpp")] + \
      [os.path.join(ROOT, "tests", "host_asan", f) for f in ("stub_hip.cpp", "batch_harness.cpp")]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    out = str(tmp_path_factory.mktemp("asan") / "batch_harness")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *SRC, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def _run(harness, lines, tmp_path):
    wl = tmp_path / "workload.txt"
    wl.write_text("".join(f"{n} {L} {E} {M} {lev}\n" for n, L, E, M, lev in lines))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([harness, str(wl)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ERROR: " not in r.stderr and "runtime error" not in r.stderr, \
        r.stdout + r.stderr[-4000:]
    assert r.stdout.strip().endswith("OK")
    return r.stdout


def test_batch_of_16_host_bookkeeping_is_memory_safe(harness, tmp_path):
    lines = [(64 if i % 2 else 128, 20.0 if i % 2 else 40.0, 0.05 + 0.11 * i, 2 + (i % 7), 4 if i % 2 else 5)
             for i in range(16)]
    out = _run(harness, lines, tmp_path)
    assert "16 handles set up" in out and "stopped at the limit" in out


def test_batch_of_64_mixed_size_host_bookkeeping_is_memory_safe(harness, tmp_path):
    lines = [(w.n, w.L, w.E, w.M, w.levels) for w in batch_workloads()]
    out = _run(harness, lines, tmp_path)
    assert "64 handles set up" in out and "24 of 64 stopped at the limit" in out
