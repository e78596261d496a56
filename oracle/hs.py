"""Alg. 2: cost, gradient and HVP of the Hilbert-Schmidt test from the
overlap and its derivatives (oracle; test infrastructure only).

Per sample s the inputs are the overlap T_s = phi_s^dag G psi_s, its complex
(holomorphic) derivative dT_s/dG_k (Eq. environment) and the directional
derivative of that derivative along V (the "HVP of the overlap", Eq.
overlap-hvp).  The cost is the empirical risk of Eq. costHS,
C = 1 - (1/N_s) sum_s |T_s|^2.

Reading of the paper's signs: Eq. grad-costHS prints the gradient of |T|^2
while Alg. 2 returns 1 - |T|^2 and Eq. hvp-costHS differentiates the
gradient of 1 - |T|^2.  The oracle returns the derivatives of the cost it
returns: grad C = +2 T grad L_F with grad L_F = -conj(dT/dG) (Eq. grad-costF),
and H(C)[V] = 2 (Omega grad L_F + T H(L_F)[V]) (Eq. hvp-costHS).  Central
finite differences of C pin this choice (tests).
"""
from __future__ import annotations

import numpy as np


def hs_outputs(T: np.ndarray, dT: np.ndarray, hT: np.ndarray | None, V: np.ndarray | None):
    """Average the per-sample Alg. 2 outputs over samples.

    T : (N_s,) complex; dT, hT : (N_s, K, 4, 4) complex; V : (K, 4, 4).
    Returns dict with cost C, fidelity F, grad (K,4,4) and, if hT is given,
    hvp (K,4,4) and Omega (N_s,).
    """
    N = T.shape[0]
    F = float(np.mean(np.abs(T) ** 2))
    out = {"cost": 1.0 - F, "fidelity": F, "T": T}
    gradLF = -np.conj(dT)                                   # Eq. grad-costF, per sample
    grad = 2.0 * T[:, None, None, None] * gradLF            # gradient of 1 - |T|^2 (sign reading above)
    out["grad"] = grad.sum(axis=0) / N
    if hT is not None:
        # Omega = -sum_k <grad_k L_F, V_k> with <A, B> = Tr(A^dag B)  (Eq. Omega, App. B)
        Omega = -np.einsum("skij,kij->s", np.conj(gradLF), V)
        hLF = -np.conj(hT)                                   # Eq. hvp-costF
        h = 2.0 * (Omega[:, None, None, None] * gradLF + T[:, None, None, None] * hLF)
        out["hvp"] = h.sum(axis=0) / N
        out["Omega"] = Omega
    return out


def inner(A: np.ndarray, B: np.ndarray) -> complex:
    """Hilbert-Schmidt inner product summed over gates: sum_k Tr(A_k^dag B_k)."""
    return complex(np.sum(np.conj(A) * B))
