"""The library's host runtime (qhvp_host.cpp) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer against a host-only stand-in for the HIP runtime
(tests/host_harness/hip_stub.cpp), and driven through pass planning and workspace layouts over many
shapes, the FP64 utilities, every argument and allocation error path of problem creation (the
library's own workspace and each pinned staging buffer failing in turn must give QHVP_ERR_NOMEM and
release everything acquired before the failure), and the call sequences of the host,
device-pointer and allocation-free entry points (tests/host_harness/driver.cpp).  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host_harness")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(HARNESS, "driver.cpp"), os.path.join(HARNESS, "hip_stub.cpp"),
           os.path.join(ROOT, "paper_2604_20384_amd", "csrc", "qhvp_host.cpp"), "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    for section in ("OK plans", "OK utilities", "OK creation errors", "OK call sequences", "ALL OK"):
        assert section in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_tile_addressing_covers_each_tile_once(tmp_path):
    """The per-gate LDS offsets the host gives the kernels (tests/host_harness/layout_check.cpp):
    for n = 2..30 and nine depths, both precisions, every gate's group and amplitude bits cover the
    tile's bits once through single-bit offsets of a one-to-one layout, and wave-local passes keep
    each wave on its own quarter of the tile."""
    exe = tmp_path / "layout_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HARNESS, "layout_check.cpp"), os.path.join(HARNESS, "hip_stub.cpp"), "-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "LAYOUT OK" in r.stdout, (r.stdout[-3000:], r.stderr[-3000:])
