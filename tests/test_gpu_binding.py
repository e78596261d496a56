"""The Python binding in a fresh process whose first GPU use is the library's.

PyTorch-ROCm carries its own HIP runtime beside the system one that libqhvp links; the binding
initialises torch's first, so a Problem can be the first thing a program creates on the GPU.  The
child process runs one small HVP and checks it against the oracle, which it computes itself.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
from paper_2604_20384_amd.inputs import make_problem
from paper_2604_20384_amd.api import Problem       # no torch call before this point
p = make_problem(8, 4, 3, seed=41)
gp = Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision="c128", ckpt_every=1)
c, g, h = gp.hvp(p.G, p.V)
gp.close()
from oracle import circuit, sv
psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
ref = sv.evaluate(psi, phi, p.G, p.V, p.n, p.L)
err = max(np.linalg.norm(g - ref["grad"]) / np.linalg.norm(ref["grad"]),
          np.linalg.norm(h - ref["hvp"]) / np.linalg.norm(ref["hvp"]))
print("child rel err", err, flush=True)
assert err <= 1e-10
"""


def test_problem_first_gpu_use_in_fresh_process(gpu):
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0
    assert "child rel err" in r.stdout
