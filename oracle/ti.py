"""Translationally invariant brickwalls (oracle; test infrastructure only).

App. E: every gate of layer l is the same matrix G_(l) (and the direction is V_(l) on all of
them); the derivative of the overlap with respect to G_(l) is the sum over the layer's gates of
the per-gate derivatives, and so are the gradient and the HVP of the cost.  The printed Alg. 3
has garbled indices; the oracle follows the prose definition: expand, evaluate per gate, sum.
"""
from __future__ import annotations

import numpy as np

from .circuit import brickwall_positions, labels
from . import sv


def expand(layer_mats: np.ndarray, n: int, L: int) -> np.ndarray:
    return np.stack([layer_mats[layer] for layer, _ in brickwall_positions(n, L)])


def reduce(per_gate: np.ndarray, n: int, L: int) -> np.ndarray:
    out = np.zeros((L, 4, 4), dtype=np.complex128)
    for k, (layer, _) in enumerate(brickwall_positions(n, L)):
        out[layer] += per_gate[k]
    return out


def evaluate(uref, samples, G_layers, V_layers, n, L, L_ref):
    psi, phi = labels(uref, samples, n, L_ref)
    G = expand(G_layers, n, L)
    V = None if V_layers is None else expand(V_layers, n, L)
    out = sv.evaluate(psi, phi, G, V, n, L)
    res = {"cost": out["cost"], "fidelity": out["fidelity"], "grad": reduce(out["grad"], n, L)}
    if V is not None:
        res["hvp"] = reduce(out["hvp"], n, L)
    return res
