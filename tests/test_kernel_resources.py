"""Resource usage of the compiled kernels (CPU only: hipcc cross-compiles the device code).

* No kernel uses private (scratch) memory: the entry point that allocates nothing relies on it (a
  kernel with scratch makes the runtime reserve memory behind the caller's back).
* The hot kernels keep the occupancy their designs are measured at: two waves per SIMD for the
  backward kernels from pass outputs (complex64 and complex128, 6-gate instances), four for the
  complex64 forward kernel.

The figures are the compiler's own resource report (-Rpass-analysis=kernel-resource-usage) for the
flags the library is built with.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2604_20384_amd import build

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2604_20384_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


def _resources(src):
    cmd = ["hipcc", f"--offload-arch={build.ARCH}", *build.DEVICE_FLAGS, "-O3", "-std=c++17", "--cuda-device-only",
           "-c", "-Rpass-analysis=kernel-resource-usage", "-o", os.devnull, os.path.join(CSRC, src)]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    info, cur = {}, None
    for line in out.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            info[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?): (\S+) \[-Rpass", line)
        if m and cur:
            info[cur][m.group(1).strip()] = m.group(2)
    return info


@pytest.fixture(scope="module")
def kernels():
    info = {}
    for src in ("qhvp_kernels.hip", "qhvp_post.hip"):
        info.update(_resources(src))
    return info


def test_no_kernel_uses_scratch(kernels):
    assert len(kernels) >= 40
    used = {k: v["ScratchSize [bytes/lane]"] for k, v in kernels.items() if v["ScratchSize [bytes/lane]"] != "0"}
    assert not used, used


@pytest.mark.parametrize("name,waves", [
    ("_ZN4qhvp9k_bwd_outIfLb1ELi6EEEvNS_7BwdArgsE", 2),   # k_bwd_out<float, true, 6>
    ("_ZN4qhvp9k_bwd_outIdLb1ELi6EEEvNS_7BwdArgsE", 2),   # k_bwd_out<double, true, 6>
    ("_ZN4qhvp5k_fwdIfLb1ELi6EEEvNS_7FwdArgsE", 4),       # k_fwd<float, true, 6>
])
def test_hot_kernel_occupancy(kernels, name, waves):
    assert int(kernels[name]["Occupancy [waves/SIMD]"]) >= waves, kernels[name]
