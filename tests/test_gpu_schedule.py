"""Tile scheduling of the forward kernel: launches with at least 16 tiles per workgroup take tiles
dynamically, in chunks from a per-launch counter; smaller launches split them statically.  The
results do not depend on the schedule: the forward kernel's outputs are per tile, and the backward
kernels keep their static split.

n=10, L=2 (tile = whole statevector), N_s = 16385 samples: 16385 tiles, dynamic at every size of
the resident grid, chunks of 4 tiles with a last chunk of one.  Checked against the oracle over all
samples (complex128 1e-10, complex64 1e-5) and bit for bit against the static split forced with
QHVP_SCHEDULE=static.
"""
import os
import numpy as np
import pytest

from oracle import circuit, sv
from parity import assert_close, assert_fidelity
from paper_2604_20384_amd.inputs import make_problem

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N, L, NS, SEED = 10, 2, 16385, 41
TOL = {"c128": 1e-10, "c64": 1e-5}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _gpu(precision):
    from paper_2604_20384_amd.api import Problem
    p = make_problem(N, L, NS, seed=SEED)
    gp = Problem(N, L, p.uref, p.samples, L_ref=p.L_ref, precision=precision, ckpt_every=0)
    out = gp.hvp(p.G, p.V)
    F = gp.last_fidelity
    T, Om = gp.overlaps()
    gp.close()
    return out, F, T, Om


@pytest.fixture(scope="module")
def oracle_ref():
    p = make_problem(N, L, NS, seed=SEED)
    psi, phi = circuit.labels(p.uref, p.samples, N, p.L_ref)
    return sv.evaluate(psi, phi, p.G, p.V, N, L, batch=4096)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_dynamic_schedule_matches_oracle_and_static_split(gpu, oracle_ref, precision):
    (c, g, h), F, T, Om = _gpu(precision)
    ref = oracle_ref
    tol = TOL[precision]
    eF = assert_fidelity(F, ref["fidelity"], tol, precision)
    eg = assert_close(g, ref["grad"], tol, precision + " grad")
    eh = assert_close(h, ref["hvp"], tol, precision + " hvp")
    print(f"n={N} L={L} N_s={NS} {precision}: rel err F {eF:.2e} grad {eg[0]:.2e} (per gate {eg[1]:.2e}) "
          f"hvp {eh[0]:.2e} (per gate {eh[1]:.2e})")
    assert np.linalg.norm(T - ref["T"]) <= tol * np.linalg.norm(ref["T"])
    # the same evaluation with the static split
    os.environ["QHVP_SCHEDULE"] = "static"
    try:
        (c2, g2, h2), F2, T2, Om2 = _gpu(precision)
    finally:
        del os.environ["QHVP_SCHEDULE"]
    assert c2 == c and np.array_equal(g2, g) and np.array_equal(h2, h)
    assert np.array_equal(T2, T) and np.array_equal(Om2, Om)
