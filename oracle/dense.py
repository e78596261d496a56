"""Brute-force derivatives of the overlap by substitution (oracle; test
infrastructure only).  No recursion, no cached intermediate states.

The overlap T_s(G) = phi_s^dag G_K ... G_1 psi_s is linear in every gate
(Sec. II.B, the holomorphic overlap), so:

* dT_s/dG_{k,ij} is T_s with gate k replaced by the unit matrix e_i e_j^T
  (Eq. environment, "cutting out" gate k);
* the directional derivative of that environment along V is the sum over
  every other gate k' != k of T_s with gate k replaced by e_i e_j^T and
  gate k' replaced by V_{k'} (Sec. III, "HVP via recursive tangent-state
  propagation": one gate replaced by its variation in each summand).  The
  k' = k term vanishes because the substituted overlap no longer depends
  on G_k.

Both are evaluated literally, one substituted circuit at a time, on the
batch of samples; this is exponential in nothing but slow (K^2 * 16
circuits), which is fine for the tiny sizes it serves (n <= 8).
"""
from __future__ import annotations

import numpy as np

from .circuit import apply_gate, brickwall_positions, dense_circuit, labels
from .hs import hs_outputs


def _unit(i: int, j: int) -> np.ndarray:
    e = np.zeros((4, 4), dtype=np.complex128)
    e[i, j] = 1.0
    return e


def substituted_overlap(psi: np.ndarray, phi: np.ndarray, gates: np.ndarray, n: int, L: int,
                        subst: dict) -> np.ndarray:
    """T_s with gate k replaced by subst[k], for psi, phi of shape (N_s, 2^n); returns (N_s,)."""
    state = psi.T.copy()
    for k, (_, q) in enumerate(brickwall_positions(n, L)):
        state = apply_gate(state, subst.get(k, gates[k]), q, n)
    return np.einsum("sx,xs->s", np.conj(phi), state)


def overlap_dense(psi, phi, gates, n, L) -> np.ndarray:
    """T_s = phi_s^dag U psi_s with U built as a dense 2^n x 2^n matrix."""
    U = dense_circuit(gates, n, L)
    return np.einsum("sx,xy,sy->s", np.conj(phi), U, psi)


def derivatives(psi, phi, gates, V, n, L):
    """(T, dT, hT) by substitution; dT, hT have shape (N_s, K, 4, 4)."""
    K = gates.shape[0]
    Ns = psi.shape[0]
    T = overlap_dense(psi, phi, gates, n, L)
    dT = np.zeros((Ns, K, 4, 4), dtype=np.complex128)
    hT = np.zeros((Ns, K, 4, 4), dtype=np.complex128) if V is not None else None
    for k in range(K):
        for i in range(4):
            for j in range(4):
                e = _unit(i, j)
                dT[:, k, i, j] = substituted_overlap(psi, phi, gates, n, L, {k: e})
                if V is not None:
                    acc = np.zeros(Ns, dtype=np.complex128)
                    for kp in range(K):
                        if kp != k:
                            acc += substituted_overlap(psi, phi, gates, n, L, {k: e, kp: V[kp]})
                    hT[:, k, i, j] = acc
    return T, dT, hT


def evaluate(uref, samples, gates, V, n, L, L_ref):
    """Cost, gradient and HVP (Alg. 2 post-processing) from the substitution derivatives."""
    psi, phi = labels(uref, samples, n, L_ref)
    T, dT, hT = derivatives(psi, phi, gates, V, n, L)
    return hs_outputs(T, dT, hT, V)
