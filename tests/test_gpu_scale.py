"""Parity and properties at the headline size n=20, L=20 (K=190), N_s=256 (U_ref depth 40).

The oracle cannot run all 256 samples in test time, so:
* the first 4 samples run through both the oracle and the GPU (a 4-sample problem, every pass
  boundary kept as in the headline run) and the fidelity / gradient / HVP are compared in
  complex128 (1e-10) and complex64 (1e-5), globally and gate by gate;
* on all 256 samples, the complex64 run (every pass boundary kept) is compared with an
  all-complex128 GPU run of the same problem (complex128 is within 1e-10 of the oracle wherever
  the oracle reaches, so it stands in for it here), globally and gate by gate;
* on the full problem, sampled per-sample overlaps T_s are checked against the oracle one sample at
  a time, and size-independent identities are checked: the Euler identity of the multilinear
  overlap, Hessian symmetry, and central differences of the fidelity (complex128).
"""
import numpy as np
import pytest

from oracle import circuit, sv
from parity import assert_close, assert_fidelity, per_gate_rel, rel
from paper_2604_20384_amd.inputs import make_problem

pytestmark = pytest.mark.gpu

N, L, NS = 20, 20, 256


@pytest.fixture(scope="module")
def prob():
    return make_problem(N, L, NS, seed=1)


def test_first_four_samples_against_oracle(gpu, prob):
    import torch

    from paper_2604_20384_amd.api import Problem
    torch.cuda.empty_cache()
    ns = 4
    psi, phi = circuit.labels(prob.uref, prob.samples[:ns], N, prob.L_ref)
    ref = sv.evaluate(psi, phi, prob.G, prob.V, N, L, batch=1)
    for precision, tol in (("c128", 1e-10), ("c64", 1e-5)):
        gp = Problem(N, L, prob.uref, prob.samples[:ns], L_ref=prob.L_ref, precision=precision, ckpt_every=0)
        c, g, h = gp.hvp(prob.G, prob.V)
        eF = assert_fidelity(gp.last_fidelity, ref["fidelity"], tol, precision)
        eg = assert_close(g, ref["grad"], tol, precision + " grad")
        eh = assert_close(h, ref["hvp"], tol, precision + " hvp")
        print(f"n=20 L=20 first {ns} samples {precision}: rel err F {eF:.2e} grad {eg[0]:.2e} "
              f"(per gate {eg[1]:.2e}) hvp {eh[0]:.2e} (per gate {eh[1]:.2e})")
        gp.close()


def test_full_size_c64_against_c128(gpu, prob):
    """Pattern (1): complex64 states with FP64 accumulation against an all-complex128 GPU run on
    all 256 samples (complex64 with every pass boundary kept, the headline setting)."""
    import torch

    from paper_2604_20384_amd.api import Problem
    out = {}
    for precision, ckpt in (("c64", 0), ("c128", 1)):
        torch.cuda.empty_cache()
        gp = Problem(N, L, prob.uref, prob.samples, L_ref=prob.L_ref, precision=precision, ckpt_every=ckpt)
        c, g, h = gp.hvp(prob.G, prob.V)
        out[precision] = (gp.last_fidelity, g, h)
        gp.close()
        del gp
    (F4, g4, h4), (F8, g8, h8) = out["c64"], out["c128"]
    eF = assert_fidelity(F4, F8, 1e-5, "c64 vs c128")
    eg = assert_close(g4, g8, 1e-5, "c64 vs c128 grad")
    eh = assert_close(h4, h8, 1e-5, "c64 vs c128 hvp")
    print(f"n=20 L=20 N_s=256 c64 vs c128: rel err F {eF:.2e} grad {eg[0]:.2e} (per gate {eg[1]:.2e}) "
          f"hvp {eh[0]:.2e} (per gate {eh[1]:.2e})")


def test_full_size_sampled_overlaps_and_identities(gpu, prob):
    import torch

    from paper_2604_20384_amd.api import Problem
    torch.cuda.empty_cache()
    gp = Problem(N, L, prob.uref, prob.samples, L_ref=prob.L_ref, precision="c64", ckpt_every=0)
    c, g, h = gp.hvp(prob.G, prob.V)
    F = gp.last_fidelity
    T, Om = gp.overlaps()
    # sampled outputs the oracle computes one sample at a time
    for s in (0, 131, 255):
        psi, phi = circuit.labels(prob.uref, prob.samples[s:s + 1], N, prob.L_ref)
        Ts = np.vdot(phi[0], circuit.apply_circuit(psi[0][:, None], prob.G, N, L)[:, 0])
        assert abs(T[s] - Ts) <= 1e-5 * abs(Ts)
    assert abs(F - np.mean(np.abs(T) ** 2)) <= 1e-12 * F
    # Euler identity: sum_ij conj(grad_k)_ij G_k,ij = -2F for every gate (T is linear in each gate)
    e = np.einsum("kij,kij->k", np.conj(g), prob.G)
    assert np.max(np.abs(e + 2 * F)) <= 1e-5 * 2 * F
    # symmetry of the Hessian: Re<W, H V> = Re<V, H W>
    rng = np.random.default_rng(0)
    W = rng.standard_normal(prob.G.shape) + 1j * rng.standard_normal(prob.G.shape)
    _, _, hW = gp.hvp(prob.G, W)
    a, b = np.vdot(W, h).real, np.vdot(prob.V, hW).real
    assert abs(a - b) <= 1e-4 * max(abs(a), abs(b))
    gp.close()


def test_full_size_finite_differences_c128(gpu, prob):
    import torch

    from paper_2604_20384_amd.api import Problem
    torch.cuda.empty_cache()
    gp = Problem(N, L, prob.uref, prob.samples, L_ref=prob.L_ref, precision="c128", ckpt_every=2)
    c, g, h = gp.hvp(prob.G, prob.V)
    hstep = 1e-6
    Fp = gp.cost(prob.G + hstep * prob.V)[1]
    Fm = gp.cost(prob.G - hstep * prob.V)[1]
    fd = -(Fp - Fm) / (2 * hstep)
    an = np.vdot(g, prob.V).real
    print(f"n=20 full size c128: FD {fd:.6e} analytic {an:.6e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
    gp.close()
