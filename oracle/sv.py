"""Alg. 1 (HVP kernel for a composition of linear maps) on full statevectors,
followed by Alg. 2 (oracle; test infrastructure only).

Forward pass: psi^[k] = G_k psi^[k-1] (Eq. fis) and the forward tangent
state dpsi^[k] = G_k dpsi^[k-1] + V_k psi^[k-1] (Eq. dfis), both cached for
every gate.  Backward pass from phi^[0] = phi (the label U_ref psi), with
the backward tangent dphi (Eq. bis, Eq. dbis), accumulating for gate k the
environment conj(phi^[K-k]) (x) psi^[k-1] (Eq. environment) and the
future + past terms of Eq. overlap-hvp.

Statement order: Alg. 1 as printed updates dphi before it is used for gate
k; that would add gate k's own variation V_k^dag phi to its HVP term,
which the definition (one gate replaced by its variation, every *other*
gate; Sec. III) excludes.  The oracle accumulates gate k's terms first and
then updates dphi and phi.  The brute-force substitution in `dense` pins
this (tests).
"""
from __future__ import annotations

import numpy as np

from .circuit import apply_gate, brickwall_positions, pair_unfold
from .hs import hs_outputs


def _env(left: np.ndarray, right: np.ndarray, q: int, n: int) -> np.ndarray:
    """sum_alpha conj(left)_{i alpha} right_{j alpha} for a batch (2^n, B) -> (B, 4, 4)."""
    B = left.shape[1]
    out = np.empty((B, 4, 4), dtype=np.complex128)
    for b in range(B):
        l = pair_unfold(left[:, b], q, n)
        r = pair_unfold(right[:, b], q, n)
        out[b] = np.conj(l) @ r.T
    return out


def hvp_kernel(psi0: np.ndarray, phi0: np.ndarray, gates: np.ndarray, V: np.ndarray | None,
               n: int, L: int, keep_states: bool = False, printed_order: bool = False):
    """Alg. 1 for a batch of samples.

    psi0, phi0 : (2^n, B) boundary states.  Returns (T (B,), dT (B,K,4,4),
    hT (B,K,4,4) or None[, states]).  `printed_order=True` updates dphi
    before gate k's HVP term, as Alg. 1 is printed; it exists only so a test
    can show that the brute force rejects that order.
    """
    pos = brickwall_positions(n, L)
    K = len(pos)
    B = psi0.shape[1]
    tangent = V is not None
    # forward pass: cache psi^[k] and dpsi^[k] for k = 0..K
    psi = [psi0]
    dpsi = [np.zeros_like(psi0)] if tangent else None
    for k, (_, q) in enumerate(pos):
        if tangent:
            dpsi.append(apply_gate(dpsi[k], gates[k], q, n) + apply_gate(psi[k], V[k], q, n))
        psi.append(apply_gate(psi[k], gates[k], q, n))
    # backward pass
    phi = phi0.copy()
    dphi = np.zeros_like(phi0) if tangent else None
    dT = np.zeros((B, K, 4, 4), dtype=np.complex128)
    hT = np.zeros((B, K, 4, 4), dtype=np.complex128) if tangent else None
    phis = [None] * K
    for k in range(K - 1, -1, -1):
        q = pos[k][1]
        if keep_states:
            phis[k] = phi.copy()
        # gate k's terms use phi^[K-k], dphi^[K-k] (gate k not yet undone) and psi^[k-1], dpsi^[k-1]
        dT[:, k] = _env(phi, psi[k], q, n)
        if tangent:
            Gd = np.conj(gates[k].T)
            Vd = np.conj(V[k].T)
            if printed_order:
                dphi = apply_gate(dphi, Gd, q, n) + apply_gate(phi, Vd, q, n)
            hT[:, k] = _env(dphi, psi[k], q, n) + _env(phi, dpsi[k], q, n)
            if not printed_order:
                dphi = apply_gate(dphi, Gd, q, n) + apply_gate(phi, Vd, q, n)
        phi = apply_gate(phi, np.conj(gates[k].T), q, n)
    T = np.einsum("xb,xb->b", np.conj(phi), psi0)          # T = phi^[K]^dag psi^[0]
    if keep_states:
        return T, dT, hT, {"psi": psi, "dpsi": dpsi, "phi_after": phis}
    return T, dT, hT


def evaluate(psi0: np.ndarray, phi0: np.ndarray, gates: np.ndarray, V: np.ndarray | None,
             n: int, L: int, batch: int = 64):
    """Alg. 2 over all samples: psi0, phi0 of shape (N_s, 2^n).  Returns the `hs_outputs` dict."""
    Ns = psi0.shape[0]
    Ts, dTs, hTs = [], [], []
    for s0 in range(0, Ns, batch):
        sl = slice(s0, min(Ns, s0 + batch))
        T, dT, hT = hvp_kernel(psi0[sl].T.copy(), phi0[sl].T.copy(), gates, V, n, L)
        Ts.append(T)
        dTs.append(dT)
        if hT is not None:
            hTs.append(hT)
    T = np.concatenate(Ts)
    dT = np.concatenate(dTs)
    hT = np.concatenate(hTs) if hTs else None
    return hs_outputs(T, dT, hT, V)
