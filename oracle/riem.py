"""Unitary-manifold geometry for gate vectors in U(4)^K (oracle; test
infrastructure only).  App. F: projection onto the tangent space, the
Riemannian gradient and the Riemannian HVP; App. G: the Pauli tangent
basis.  The paper names no retraction; the oracle uses the polar one,
R_G(xi) = the unitary factor of G + xi, which is one valid choice (parity
unpinned as a choice; pinned by its defining properties in the tests).
"""
from __future__ import annotations

import numpy as np


def dag(A: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(A, -1, -2))


def project(G: np.ndarray, X: np.ndarray) -> np.ndarray:
    """P_G(X) = G skew(G^dag X) = X/2 - G X^dag G / 2, gate by gate (Eq. projec)."""
    return 0.5 * X - 0.5 * G @ dag(X) @ G


def riemannian_grad(G: np.ndarray, egrad: np.ndarray) -> np.ndarray:
    """grad_R f = [P_{G_k}(grad_k f)]_k (App. F)."""
    return project(G, egrad)


def riemannian_hvp(G: np.ndarray, egrad: np.ndarray, ehvp: np.ndarray, V: np.ndarray) -> np.ndarray:
    """H_R(f)[V] = P_G(H(f)[V] - V grad^dag G / 2 - G grad^dag V / 2), gate by gate (App. F).

    The formula is derived for a tangent V; callers project V first.
    """
    inner = ehvp - 0.5 * V @ dag(egrad) @ G - 0.5 * G @ dag(egrad) @ V
    return project(G, inner)


def retract(G: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Polar retraction: the unitary polar factor U W^dag of G + xi = U S W^dag."""
    A = G + xi
    U, _, Wh = np.linalg.svd(A)
    return U @ Wh


_PAULI = [np.eye(2, dtype=np.complex128),
          np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def pauli_tangent_basis(Gk: np.ndarray) -> np.ndarray:
    """{i G (P_a (x) P_b) / 2}: 16 tangent vectors at G, orthonormal under Re Tr(A^dag B) (App. G)."""
    out = np.empty((16, 4, 4), dtype=np.complex128)
    for a in range(4):
        for b in range(4):
            out[4 * a + b] = 0.5j * Gk @ np.kron(_PAULI[a], _PAULI[b])
    return out
