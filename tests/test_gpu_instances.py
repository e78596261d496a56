"""Every complex64 kernel instance against the oracle.

complex64 compiles the forward and backward kernels once per pass gate count (1..6).  Each case
below is a shape whose pass plan contains the listed gate counts (asserted, so the case keeps its
meaning if the planner changes), run as a complex64 HVP and compared with the oracle; small tiles
(n = 2, 5, 6: one tile per sample, workgroup barriers between gates) and full wave-local tiles
(n >= 11).
"""
import pytest

from oracle import circuit, sv
from paper_2604_20384_amd.api import plan
from paper_2604_20384_amd.inputs import make_problem
from parity import assert_close, assert_fidelity

pytestmark = pytest.mark.gpu

CASES = [  # (n, L, N_s, gate counts its ansatz plan must contain)
    (2, 1, 3, {1}), (6, 3, 3, {2, 6}), (2, 5, 3, {3}), (2, 7, 3, {4}), (2, 9, 3, {5}),
    (13, 11, 2, {1, 5, 6}), (13, 3, 2, {2, 4, 6}), (12, 7, 2, {3, 6}),
]


@pytest.mark.parametrize("n,L,ns,counts", CASES)
def test_c64_instances_against_oracle(gpu, n, L, ns, counts):
    from paper_2604_20384_amd.api import Problem
    per, _ = plan(n, L)
    assert counts <= set(per), (n, L, per)
    p = make_problem(n, L, ns, seed=50 + n + L)
    psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
    ref = sv.evaluate(psi, phi, p.G, p.V, p.n, p.L)
    for ckpt in (0, 1):
        gp = Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision="c64", ckpt_every=ckpt)
        c, g, h = gp.hvp(p.G, p.V)
        F = gp.last_fidelity
        assert gp.backward_from_outputs
        gp.close()
        assert_fidelity(F, ref["fidelity"], 1e-5, (n, L, ckpt))
        assert_close(g, ref["grad"], 1e-5, (n, L, ckpt, "grad"))
        assert_close(h, ref["hvp"], 1e-5, (n, L, ckpt, "hvp"))
