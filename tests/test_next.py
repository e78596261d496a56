"""Rows beyond the core path: translationally invariant circuits (App. E), the dense Riemannian
Hessian in the Pauli basis (App. G), and the Riemannian trust-region / truncated-CG driver."""
import numpy as np
import pytest

from oracle import circuit, dense, hs, riem, sv, ti
from parity import assert_close, assert_fidelity
from paper_2604_20384_amd import hessian, optim
from paper_2604_20384_amd.inputs import haar_unitary, make_problem, random_antihermitian


class OracleModel:
    """cost / grad / hvp (Euclidean or Riemannian) from the CPU oracle; test-only."""

    def __init__(self, p, n_samples=None):
        self.p = p
        ns = p.n_samples if n_samples is None else n_samples
        self.psi, self.phi = circuit.labels(p.uref, p.samples[:ns], p.n, p.L_ref)

    def _ev(self, G, V):
        return sv.evaluate(self.psi, self.phi, G, V, self.p.n, self.p.L)

    def cost(self, G):
        o = self._ev(G, None)
        return o["cost"], o["fidelity"]

    def grad(self, G, riemannian=False):
        o = self._ev(G, None)
        return o["cost"], (riem.riemannian_grad(G, o["grad"]) if riemannian else o["grad"])

    def hvp(self, G, V, riemannian=False):
        if riemannian:
            V = riem.project(G, V)
        o = self._ev(G, V)
        if not riemannian:
            return o["cost"], o["grad"], o["hvp"]
        return o["cost"], riem.riemannian_grad(G, o["grad"]), riem.riemannian_hvp(G, o["grad"], o["hvp"], V)


def _ti_problem(n, L, ns, seed):
    p = make_problem(n, L, ns, seed=seed)
    rng = np.random.default_rng(seed + 1)
    Gl = haar_unitary(rng, 4, L)
    Vl = Gl @ random_antihermitian(rng, L)
    return p, Gl, Vl


# ---------------------------------------------------------------------------------------------
# CPU: pins of the oracle-side definitions

def test_ti_oracle_finite_differences():
    """The per-layer gradient / HVP are the derivatives of C(G_(1..L)) with shared layer gates."""
    n, L = 5, 4
    p, Gl, Vl = _ti_problem(n, L, 3, 10)
    rng = np.random.default_rng(0)
    D = rng.standard_normal(Gl.shape) + 1j * rng.standard_normal(Gl.shape)
    out = ti.evaluate(p.uref, p.samples, Gl, D, n, L, p.L_ref)
    psi, phi = circuit.labels(p.uref, p.samples, n, p.L_ref)
    h = 1e-6

    def F(Glayers):
        return np.mean(np.abs(dense.substituted_overlap(psi, phi, ti.expand(Glayers, n, L), n, L, {})) ** 2)

    fd = -(F(Gl + h * D) - F(Gl - h * D)) / (2 * h)
    assert abs(fd - hs.inner(out["grad"], D).real) < 1e-8
    h2 = 1e-5
    gp = ti.evaluate(p.uref, p.samples, Gl + h2 * D, None, n, L, p.L_ref)["grad"]
    gm = ti.evaluate(p.uref, p.samples, Gl - h2 * D, None, n, L, p.L_ref)["grad"]
    assert np.linalg.norm((gp - gm) / (2 * h2) - out["hvp"]) <= 1e-7 * np.linalg.norm(out["hvp"])


def test_pauli_basis_matches_oracle_and_is_orthonormal():
    rng = np.random.default_rng(1)
    G = haar_unitary(rng, 4, 3)
    E = hessian.tangent_basis(G)
    gram = np.real(np.einsum("ikab,jkab->ij", np.conj(E), E))
    assert np.allclose(gram, np.eye(48), atol=1e-14)
    for k in range(3):
        assert np.allclose(E[16 * k:16 * k + 16, k], riem.pauli_tangent_basis(G[k]), atol=1e-15)


def test_dense_hessian_with_oracle_is_symmetric_and_psd_at_optimum():
    p = make_problem(4, 2, 4, seed=5, L_ref=2)
    m = OracleModel(p)
    H = hessian.riemannian_hessian(lambda g, v: m.hvp(g, v, riemannian=True)[2], p.uref)
    assert np.allclose(H, H.T, atol=1e-13)
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > -1e-12


def test_trust_region_with_oracle_model_converges():
    p = make_problem(4, 2, 4, seed=6, L_ref=2)
    rng = np.random.default_rng(2)
    G0 = riem.retract(p.uref, 0.3 * p.uref @ random_antihermitian(rng, p.K))
    G, hist = optim.trust_region(OracleModel(p), G0, riem.retract, radius=0.5, max_iter=40, grad_tol=1e-10)
    acc = [c for c, a in zip(hist.cost[1:], hist.accepted) if a]
    assert all(b <= a + 1e-15 for a, b in zip([hist.cost[0]] + acc, acc))     # monotone
    assert hist.cost[-1] < 1e-12 and hist.grad_norm[-1] < 1e-7


# ---------------------------------------------------------------------------------------------
# GPU

@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("c128", 1e-10), ("c64", 1e-5)])
def test_ti_parity(gpu, precision, tol):
    from paper_2604_20384_amd.api import Problem
    n, L = 11, 5
    p, Gl, Vl = _ti_problem(n, L, 4, 20)
    ref = ti.evaluate(p.uref, p.samples, Gl, Vl, n, L, p.L_ref)
    gp = Problem(n, L, p.uref, p.samples, L_ref=p.L_ref, precision=precision)
    c, g, h = gp.hvp_ti(Gl, Vl)
    assert_fidelity(gp.last_fidelity, ref["fidelity"], tol, "TI")
    assert_close(g, ref["grad"], tol, "TI grad")
    assert_close(h, ref["hvp"], tol, "TI hvp")
    c2, g2 = gp.grad_ti(Gl, riemannian=True)
    assert_close(g2, riem.riemannian_grad(Gl, ref["grad"]), tol, "TI Riemannian grad")
    c3, gR, hR = gp.hvp_ti(Gl, Vl, riemannian=True)
    hR_ref = riem.riemannian_hvp(Gl, ref["grad"], ref["hvp"], Vl)
    assert_close(hR, hR_ref, tol, "TI Riemannian hvp")


@pytest.mark.gpu
def test_dense_hessian_parity(gpu):
    from paper_2604_20384_amd.api import Problem
    p = make_problem(5, 3, 3, seed=7)
    gp = Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision="c128")
    H = hessian.problem_hessian(gp, p.G)
    m = OracleModel(p)
    Href = hessian.riemannian_hessian(lambda g, v: m.hvp(g, v, riemannian=True)[2], p.G)
    assert np.linalg.norm(H - Href) <= 1e-10 * np.linalg.norm(Href)
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())


@pytest.mark.gpu
def test_trust_region_gpu_matches_oracle_iterates(gpu):
    from paper_2604_20384_amd import api
    p = make_problem(6, 2, 4, seed=8, L_ref=2)
    rng = np.random.default_rng(3)
    G0 = riem.retract(p.uref, 0.3 * p.uref @ random_antihermitian(rng, p.K))
    gp = api.Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision="c128")
    Gg, hg = optim.trust_region(gp, G0, api.retract, radius=0.5, max_iter=6)
    Go, ho = optim.trust_region(OracleModel(p), G0, riem.retract, radius=0.5, max_iter=6)
    assert hg.accepted == ho.accepted and hg.inner_iterations == ho.inner_iterations
    assert np.allclose(hg.cost, ho.cost, rtol=1e-9, atol=1e-13)
    assert np.linalg.norm(Gg - Go) <= 1e-8
    Gf, hf = optim.trust_region(gp, G0, api.retract, radius=0.5, max_iter=40, grad_tol=1e-10)
    assert hf.cost[-1] < 1e-10
