"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: complex128 -> relative error <= 1e-10; complex64 with FP64 accumulation
-> <= 1e-5.  Relative errors: |dF| / F for the fidelity (C ~ 1 - O(2^-n) makes a
relative error on C vacuous); for the gradient and the HVP both ||d|| / ||ref||
over all K*16 entries and, gate by gate, max |d_k| / max |ref_k| (tests/parity.py).
"""
import numpy as np
import pytest

from oracle import circuit, dense, riem, sv
from paper_2604_20384_amd.inputs import make_problem
from parity import assert_close, assert_fidelity

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}


def _oracle(p, V=None, n_samples=None):
    ns = p.n_samples if n_samples is None else n_samples
    psi, phi = circuit.labels(p.uref, p.samples[:ns], p.n, p.L_ref)
    return sv.evaluate(psi, phi, p.G, p.V if V is None else V, p.n, p.L)


def _gpu_problem(p, precision, ckpt_every=1, n_samples=None, with_tangent=True):
    from paper_2604_20384_amd.api import Problem
    ns = p.n_samples if n_samples is None else n_samples
    return Problem(p.n, p.L, p.uref, p.samples[:ns], L_ref=p.L_ref, precision=precision,
                   ckpt_every=ckpt_every, with_tangent=with_tangent)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check(gp, ref, precision, G, V, what=""):
    tol = TOL[precision]
    c, g, h = gp.hvp(G, V)
    F = gp.last_fidelity
    assert_fidelity(F, ref["fidelity"], tol, what)
    assert abs((1 - c) - F) <= 1e-15
    assert_close(g, ref["grad"], tol, what + " grad")
    assert_close(h, ref["hvp"], tol, what + " hvp")
    T, Om = gp.overlaps()
    assert np.linalg.norm(T - ref["T"]) <= tol * np.linalg.norm(ref["T"])
    assert np.linalg.norm(Om - ref["Omega"]) <= tol * np.linalg.norm(ref["Omega"])
    # cost and gradient through their own entry points
    c2, F2 = gp.cost(G)
    assert_fidelity(F2, ref["fidelity"], tol, what + " cost")
    c3, g3 = gp.grad(G)
    assert_close(g3, ref["grad"], tol, what + " grad call")
    assert abs(gp.last_fidelity - F) <= tol * F   # the gradient call's own fidelity
    return g, h


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_tiny_config_vs_substitution_oracle(gpu, precision):
    """n=6, L=4 (K=10), U_ref depth 8, N_s=8: against the brute-force substitution oracle too."""
    p = make_problem(6, 4, 8, seed=1)
    ref = _oracle(p)
    ref_dense = dense.evaluate(p.uref, p.samples, p.G, p.V, p.n, p.L, p.L_ref)
    assert np.allclose(ref["hvp"], ref_dense["hvp"], atol=1e-13)
    gp = _gpu_problem(p, precision)
    _check(gp, ref, precision, p.G, p.V, "C1")


SHAPES = [(2, 1, 3), (2, 4, 5), (3, 2, 4), (3, 5, 2), (4, 3, 7), (5, 6, 3), (7, 3, 5), (8, 4, 2), (9, 5, 3),
          (10, 4, 3), (11, 3, 2), (12, 5, 3), (13, 2, 2), (14, 3, 2)]


@pytest.mark.parametrize("n,L,ns", SHAPES)
def test_shapes_c128(gpu, n, L, ns):
    """Every tile shape the planner makes: n below, at and above the tile size, odd and even n,
    several passes per layer, ragged sample counts."""
    p = make_problem(n, L, ns, seed=100 + n * 7 + L)
    ref = _oracle(p)
    gp = _gpu_problem(p, "c128")
    _check(gp, ref, "c128", p.G, p.V, f"n={n} L={L}")


@pytest.mark.parametrize("n,L,ns", SHAPES)
def test_shapes_c64(gpu, n, L, ns):
    """The same shapes in complex64 (its own lane-bit choice per gate and its own LDS layout)."""
    p = make_problem(n, L, ns, seed=200 + n * 7 + L)
    ref = _oracle(p)
    gp = _gpu_problem(p, "c64")
    _check(gp, ref, "c64", p.G, p.V, f"n={n} L={L}")


@pytest.mark.parametrize("ckpt", [0, 1, 2, 3, 100, -1, -2, -5])
def test_checkpoint_schedules_are_bitwise_identical(gpu, ckpt):
    """Layer checkpointing only changes what is stored and recomputed, not the arithmetic."""
    p = make_problem(12, 7, 3, seed=33)
    base = _gpu_problem(p, "c128", ckpt_every=1)
    c0, g0, h0 = base.hvp(p.G, p.V)
    gp = _gpu_problem(p, "c128", ckpt_every=ckpt)
    c1, g1, h1 = gp.hvp(p.G, p.V)
    assert c0 == c1 and np.array_equal(g0, g1) and np.array_equal(h0, h1)


def test_repeatable_bitwise(gpu):
    p = make_problem(13, 5, 6, seed=44)
    gp = _gpu_problem(p, "c64")
    r = [gp.hvp(p.G, p.V) for _ in range(3)]
    for c, g, h in r[1:]:
        assert c == r[0][0] and np.array_equal(g, r[0][1]) and np.array_equal(h, r[0][2])


def test_non_unitary_point_and_general_direction(gpu):
    """The Euclidean formulas hold for any 4x4 matrices (the overlap is multilinear)."""
    p = make_problem(9, 4, 3, seed=55)
    rng = np.random.default_rng(5)
    G = p.G + 0.3 * (rng.standard_normal(p.G.shape) + 1j * rng.standard_normal(p.G.shape))
    V = rng.standard_normal(p.G.shape) + 1j * rng.standard_normal(p.G.shape)
    psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
    ref = sv.evaluate(psi, phi, G, V, p.n, p.L)
    gp = _gpu_problem(p, "c128")
    _check(gp, ref, "c128", G, V, "nonunitary")


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("kind", ["unitary", "near_unitary", "ill_conditioned"])
def test_backward_algorithms(gpu, monkeypatch, precision, kind):
    """The backward sweep from pass outputs (undoing gates with G^-1, environments mapped back on the
    host) and the recomputing sweep both match the oracle; near-unitary gates make G^-1 differ from
    G^dag, and gates far from unitary must fall back to recomputation."""
    p = make_problem(11, 4, 3, seed=66)
    rng = np.random.default_rng(6)
    noise = rng.standard_normal(p.G.shape) + 1j * rng.standard_normal(p.G.shape)
    G = {"unitary": p.G, "near_unitary": p.G + 0.05 * noise, "ill_conditioned": p.G + 2.0 * noise}[kind]
    V = p.V
    psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
    ref = sv.evaluate(psi, phi, G, V, p.n, p.L)
    gp = _gpu_problem(p, precision)
    monkeypatch.setenv("QHVP_BACKWARD", "recompute")
    g_r, h_r = _check(gp, ref, precision, G, V, kind + " recompute")
    assert not gp.backward_from_outputs
    monkeypatch.delenv("QHVP_BACKWARD")
    g_i, h_i = _check(gp, ref, precision, G, V, kind + " auto")
    assert gp.backward_from_outputs == (kind != "ill_conditioned")
    tol = TOL[precision]
    assert_close(g_i, g_r, tol, kind + " grad inverse vs recompute")
    assert_close(h_i, h_r, tol, kind + " hvp inverse vs recompute")


def test_riemannian_outputs(gpu):
    p = make_problem(8, 5, 4, seed=66)
    rng = np.random.default_rng(6)
    V = rng.standard_normal(p.G.shape) + 1j * rng.standard_normal(p.G.shape)   # not tangent
    gp = _gpu_problem(p, "c128")
    c, gR, hR = gp.hvp(p.G, V, riemannian=True)
    Vt = riem.project(p.G, V)
    ref = _oracle(p, V=Vt)
    assert_close(gR, riem.riemannian_grad(p.G, ref["grad"]), 1e-10, "riemannian grad")
    assert_close(hR, riem.riemannian_hvp(p.G, ref["grad"], ref["hvp"], Vt), 1e-10, "riemannian hvp")
    c2, gR2 = gp.grad(p.G, riemannian=True)
    assert_close(gR2, riem.riemannian_grad(p.G, ref["grad"]), 1e-10, "riemannian grad call")


def test_gpu_scale_config(gpu):
    """n=16, L=12 (K=90), U_ref depth 24, N_s=64, complex128 and complex64 against the oracle."""
    p = make_problem(16, 12, 64, seed=2)
    ref = _oracle(p)
    for precision in ("c128", "c64"):
        gp = _gpu_problem(p, precision)
        _check(gp, ref, precision, p.G, p.V, "C2 " + precision)
        gp.close()


def test_errors(gpu):
    from paper_2604_20384_amd._lib import QhvpError
    from paper_2604_20384_amd.api import Problem
    p = make_problem(6, 3, 2, seed=7)
    gp = _gpu_problem(p, "c128", with_tangent=False)
    gp.grad(p.G)
    with pytest.raises(QhvpError, match="UNSUPPORTED"):
        gp.hvp(p.G, p.V)
    G = p.G.copy()
    G[1, 2, 3] = np.nan
    with pytest.raises(QhvpError, match="INVALID"):
        gp.cost(G)
    with pytest.raises(QhvpError, match="INVALID"):
        gp.grad(p.G + 0.1, riemannian=True)      # Riemannian needs unitary gates
    with pytest.raises(ValueError):
        Problem(6, 3, p.uref, p.samples[:, :5], L_ref=p.L_ref)
