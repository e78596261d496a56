"""The pass planner (host logic, no device): passes of several brickwall layers must apply every
gate exactly once, each after the gates of the previous layer on overlapping qubits, so that the
planned order computes the same circuit as the layer order."""
import numpy as np
import pytest

from oracle import circuit
from paper_2604_20384_amd.inputs import haar_unitary


def _plan(n, L):
    from paper_2604_20384_amd import api
    return api.plan(n, L)


@pytest.mark.parametrize("n,L", [(2, 1), (2, 5), (3, 4), (5, 3), (6, 4), (9, 7), (10, 4), (12, 5), (16, 12),
                                 (20, 20), (23, 6), (30, 3)])
def test_plan_is_a_dependency_respecting_permutation(n, L):
    per, order = _plan(n, L)
    pos = circuit.brickwall_positions(n, L)   # gate k -> (layer, q)
    K = len(pos)
    assert sorted(order) == list(range(K)) and sum(per) == K
    assert all(1 <= c <= 6 for c in per)
    when = {k: i for i, k in enumerate(order)}
    for k, (l, q) in enumerate(pos):
        for k2, (l2, q2) in enumerate(pos):
            if l2 == l - 1 and abs(q2 - q) <= 1:   # previous layer, overlapping qubits
                assert when[k2] < when[k], (n, L, k, k2)


@pytest.mark.parametrize("n,L", [(10, 6), (12, 5), (16, 12), (20, 20), (23, 6)])
def test_plan_passes_fit_wave_local_tiles(n, L):
    """Full tiles (n >= 10): a pass spans the 4 coalesced low statevector bits plus one window of 6
    consecutive bits, and touches at most 8 of those 10, so that two untouched tile bits can index
    the waves (wave-local passes).  Gate k on qubits (q, q+1) acts on bits n-2-q and n-1-q."""
    per, order = _plan(n, L)
    pos = circuit.brickwall_positions(n, L)
    i = 0
    for c in per:
        bits = set()
        for k in order[i:i + c]:
            q = pos[k][1]
            bits |= {n - 2 - q, n - 1 - q}
        i += c
        assert len(bits) <= 8, (n, L, sorted(bits))
        high = sorted(b for b in bits if b >= 4)
        assert not high or high[-1] - high[0] < 6, (n, L, sorted(bits))


def test_plan_sizes():
    """Several layers per pass: n=20, L=20 (190 gates) takes 32 passes, the fewest at 6 gates per pass
    (one layer per pass would need 60); n=16, L=12 (90 gates) takes 15, also the fewest."""
    per, _ = _plan(20, 20)
    assert len(per) == 32 and sum(per) == 190 and max(per) <= 6
    per, _ = _plan(16, 12)
    assert len(per) == 15 and sum(per) == 90


@pytest.mark.parametrize("n,L", [(7, 6), (10, 5)])
def test_planned_order_computes_the_same_circuit(n, L):
    rng = np.random.default_rng(n * 31 + L)
    pos = circuit.brickwall_positions(n, L)
    G = haar_unitary(rng, 4, len(pos))
    psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    ref = circuit.apply_circuit(psi[:, None], G, n, L)[:, 0]
    _, order = _plan(n, L)
    out = psi.copy()
    for k in order:
        out = circuit.apply_gate(out[:, None], G[k], pos[k][1], n)[:, 0]
    assert np.allclose(out, ref, atol=1e-12)


def test_plan_rejects_bad_shapes():
    from paper_2604_20384_amd import _lib
    assert _lib.lib.qhvp_plan(1, 3, 0, None, None) < 0
    assert _lib.lib.qhvp_plan(31, 3, 0, None, None) < 0
    assert _lib.lib.qhvp_plan(20, 20, 3, (_lib.C.c_int * 3)(), None) < 0


def _header_constants(prec="C64"):
    """kLdsPad<prec> / kTsp<prec> / kMaxTileBits as written in the kernels' shared header."""
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "paper_2604_20384_amd", "csrc", "qhvp_internal.h")).read()
    pads = [int(x) for x in
            re.search(r"kLdsPad" + prec + r"\[kMaxTileBits\]\s*=\s*\{([^}]*)\}", text).group(1).split(",")]
    tsp = int(re.search(r"constexpr int kTsp" + prec + r"\s*=\s*(\d+);", text).group(1))
    bits = int(re.search(r"constexpr int kMaxTileBits\s*=\s*(\d+);", text).group(1))
    return pads, tsp, bits


def test_complex64_lds_layout_is_one_to_one():
    """The padded complex64 tile layout must give every tile element its own LDS slot below the
    second state array's offset, leave bits 0..4 unpadded (the 8- and 16-byte tile transfers read
    consecutive elements) and keep slot 32 free for the kernels' dummy writes of small tiles."""
    pads, tsp, bits = _header_constants()
    assert len(pads) == bits and pads[:5] == [0] * 5
    at = [t + sum(pads[b] for b in range(bits) if t >> b & 1) for t in range(1 << bits)]
    assert len(set(at)) == len(at)
    assert max(at) < tsp
    assert 32 not in at


def test_complex128_lds_layout_is_one_to_one():
    """The padded complex128 tile layout: one slot per tile element below the second state array's
    offset, bits 0..3 unpadded (16 lanes move 16 consecutive elements), the dummy slot free, and two
    state arrays of both tile buffers of the backward kernel within half of the 160 KB of LDS, so
    that two workgroups share a CU."""
    import re
    pads, tsp, bits = _header_constants("C128")
    assert len(pads) == bits and pads[:4] == [0] * 4
    at = [t + sum(pads[b] for b in range(bits) if t >> b & 1) for t in range(1 << bits)]
    assert len(set(at)) == len(at)
    assert max(at) < tsp
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "paper_2604_20384_amd", "csrc", "qhvp_internal.h")).read()
    dummy = int(re.search(r"constexpr int kDummyC128\s*=\s*(\d+);", text).group(1))
    assert dummy not in at and dummy < tsp
    assert 2 * 2 * tsp * 16 <= 80 * 1024 - 2048
