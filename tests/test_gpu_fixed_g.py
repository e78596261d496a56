"""Fixed-G reuse of the forward states, and HVPs along several directions at one G.

A gradient or HVP sweep leaves the forward states psi at the pass boundaries kept in the workspace,
tagged with the gates that produced them; a later gradient / HVP call at bitwise the same G stores
only the tangent states over them.  Every result must equal, bit for bit, that of a problem that
has just computed them from scratch (the same kernels read the same psi), and the oracle within the
precision's bar.  Covered: one segment (every pass boundary kept) and several (checkpoints kept,
in-segment boundaries recomputed), both backward algorithms, Euclidean and Riemannian outputs, and
calls at other gates in between.
"""
import numpy as np
import pytest

from oracle import circuit, sv
from parity import assert_close, assert_fidelity
from paper_2604_20384_amd.inputs import haar_unitary, make_problem, random_tangent

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}


def _gpu_problem(p, precision, ckpt_every):
    from paper_2604_20384_amd.api import Problem
    return Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision=precision, ckpt_every=ckpt_every)


def _fresh_hvp(p, precision, ckpt_every, G, V, riemannian=False):
    gp = _gpu_problem(p, precision, ckpt_every)
    out = gp.hvp(G, V, riemannian=riemannian)
    gp.close()
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision,ckpt", [("c64", 0), ("c64", 1), ("c128", 0), ("c128", -2)])
def test_batch_equals_fresh_single_calls(gpu, precision, ckpt):
    p = make_problem(11, 6, 5, seed=31)
    rng = np.random.default_rng(7)
    Vs = np.stack([random_tangent(rng, p.G) for _ in range(3)])
    gp = _gpu_problem(p, precision, ckpt)
    assert not gp.states_kept_for(p.G)
    c, g, H = gp.hvp_batch(p.G, Vs)
    assert gp.states_kept_for(p.G)
    print(f"batch {precision} ckpt {ckpt}: passes {gp.info()['n_passes']} segments {gp.info()['segments']}")
    for m in range(3):
        cm, gm, hm = _fresh_hvp(p, precision, ckpt, p.G, Vs[m])
        assert cm == c
        assert np.array_equal(gm, g)
        assert np.array_equal(hm, H[m]), m
    psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
    ref = sv.evaluate(psi, phi, p.G, Vs[2], p.n, p.L)
    assert_close(g, ref["grad"], TOL[precision], "fixed-G grad")
    assert_close(H[2], ref["hvp"], TOL[precision], "fixed-G hvp")
    # a second batch at the same G finds the states kept from the first one
    c2, g2, H2 = gp.hvp_batch(p.G, Vs[::-1])
    assert c2 == c and np.array_equal(g2, g) and np.array_equal(H2, H[::-1])
    gp.close()


def test_riemannian_batch_equals_fresh_calls(gpu):
    p = make_problem(9, 5, 4, seed=32)
    rng = np.random.default_rng(8)
    Vs = np.stack([random_tangent(rng, p.G) for _ in range(2)])
    gp = _gpu_problem(p, "c64", 0)
    c, g, H = gp.hvp_batch(p.G, Vs, riemannian=True)
    for m in range(2):
        cm, gm, hm = _fresh_hvp(p, "c64", 0, p.G, Vs[m], riemannian=True)
        assert np.array_equal(gm, g) and np.array_equal(hm, H[m])
    gp.close()


@pytest.mark.parametrize("ckpt", [0, 1])
def test_kept_states_follow_the_gates(gpu, ckpt):
    """Calls at other gates in between: a cost call leaves the kept states alone, a gradient or HVP
    call retags them; results at G stay those of a fresh problem throughout."""
    p = make_problem(10, 5, 4, seed=33)
    rng = np.random.default_rng(9)
    G2 = haar_unitary(rng, 4, p.K)
    V2 = random_tangent(rng, G2)
    ref = _fresh_hvp(p, "c64", ckpt, p.G, p.V)
    gp = _gpu_problem(p, "c64", ckpt)
    gp.grad(p.G)
    assert gp.states_kept_for(p.G)
    gp.cost(G2)
    assert gp.states_kept_for(p.G) and not gp.states_kept_for(G2)
    c, g, h = gp.hvp(p.G, p.V)
    assert c == ref[0] and np.array_equal(g, ref[1]) and np.array_equal(h, ref[2])
    gp.hvp(G2, V2)
    assert gp.states_kept_for(G2) and not gp.states_kept_for(p.G)
    c, g, h = gp.hvp(p.G, p.V)
    assert c == ref[0] and np.array_equal(g, ref[1]) and np.array_equal(h, ref[2])
    # the gradient through its own entry point at the kept G
    _, g3 = gp.grad(p.G)
    assert np.array_equal(g3, ref[1])
    gp.close()


def test_ill_conditioned_gates_reuse_with_recomputing_backward(gpu):
    """Gates too ill-conditioned to undo: the backward recomputes from pass inputs, also with kept
    states and several segments."""
    p = make_problem(10, 6, 3, seed=34)
    G = p.G.copy()
    G[:, :, 3] *= 10.0                       # |G|_F |G^-1|_F > 8 for every gate
    rng = np.random.default_rng(10)
    Vs = np.stack([random_tangent(rng, p.G) for _ in range(2)])
    for ckpt in (0, 1):
        gp = _gpu_problem(p, "c128", ckpt)
        c, g, H = gp.hvp_batch(G, Vs)
        assert not gp.backward_from_outputs
        for m in range(2):
            cm, gm, hm = _fresh_hvp(p, "c128", ckpt, G, Vs[m])
            assert np.array_equal(gm, g) and np.array_equal(hm, H[m])
        gp.close()


def test_reuse_stores_only_tangents(gpu):
    """With one segment every non-final forward pass of an HVP at the kept G writes S bytes fewer
    (S = one state set); the results do not change."""
    p = make_problem(12, 6, 4, seed=35)
    gp = _gpu_problem(p, "c64", 0)
    S = p.n_samples * 2 ** p.n * 8
    n_pass = gp.info()["n_passes"]
    gp.set_profiling(True)
    c1, g1, h1 = gp.hvp(p.G, p.V)
    b1 = gp.kernel_stats()["forward"]["bytes"]
    gp.set_profiling(True)
    c2, g2, h2 = gp.hvp(p.G, p.V)
    b2 = gp.kernel_stats()["forward"]["bytes"]
    assert b1 - b2 == (n_pass - 1) * S
    assert c1 == c2 and np.array_equal(g1, g2) and np.array_equal(h1, h2)
    gp.close()


def test_batch_rejects_bad_arguments(gpu):
    from paper_2604_20384_amd._lib import QhvpError
    p = make_problem(6, 3, 2, seed=36)
    gp = _gpu_problem(p, "c64", 0)
    with pytest.raises(ValueError):
        gp.hvp_batch(p.G, np.zeros((0, p.K, 4, 4)))
    bad = np.stack([p.V, p.V])
    bad[1, 0, 0, 0] = np.nan
    with pytest.raises(QhvpError):
        gp.hvp_batch(p.G, bad)
    assert not gp.states_kept_for(p.G)     # validated before any device work
    gp.close()
