"""Dense Riemannian Hessian of the Hilbert-Schmidt cost in the Pauli tangent basis (App. G).

The tangent space of U(4) at G is spanned by {i G (P_a (x) P_b) / 2 : a, b in {I, X, Y, Z}}, which
is orthonormal for the metric Re Tr(A^dag B); with one such set per gate the 16 K vectors E_i form
an orthonormal basis of the tangent space of U(4)^K, and the matrix of the Riemannian Hessian is
H_ij = Re <E_i, H_R[E_j]>, one column per Riemannian HVP.  The result is symmetric up to rounding
(the Riemannian Hessian is self-adjoint), so its spectrum is real.
"""
from __future__ import annotations

import numpy as np

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI2 = np.array([np.kron(a, b) for a in (_I, _X, _Y, _Z) for b in (_I, _X, _Y, _Z)])   # (16, 4, 4)


def tangent_basis(G: np.ndarray) -> np.ndarray:
    """(16K, K, 4, 4): basis vector 16k + m is i G_k P_m / 2 on gate k, zero elsewhere."""
    K = G.shape[0]
    E = np.zeros((16 * K, K, 4, 4), dtype=np.complex128)
    for k in range(K):
        E[16 * k:16 * k + 16, k] = 0.5j * G[k][None] @ PAULI2
    return E


def riemannian_hessian(hvp_fn, G: np.ndarray, batch_fn=None, batch: int = 64) -> np.ndarray:
    """Dense (16K x 16K) matrix from `hvp_fn(G, V) -> H_R[V]` (Riemannian HVP) on the basis, or from
    `batch_fn(G, Vs) -> H_R[Vs]` on `batch` basis vectors at a time when given."""
    E = tangent_basis(G)
    n = E.shape[0]
    H = np.empty((n, n))
    for j0 in range(0, n, batch if batch_fn is not None else 1):
        if batch_fn is not None:
            HV = batch_fn(G, E[j0:j0 + batch])
        else:
            HV = hvp_fn(G, E[j0])[None]
        for i, hv in enumerate(HV):
            H[:, j0 + i] = np.real(np.einsum("ikab,kab->i", np.conj(E), hv))
    return H


def problem_hessian(problem, G: np.ndarray, batch: int = 64) -> np.ndarray:
    """Riemannian Hessian of a `api.Problem` at unitary gates G; the columns are HVPs at one G, taken
    `batch` directions per call so that the forward states at G are computed once."""
    return riemannian_hessian(None, G, batch_fn=lambda g, vs: problem.hvp_batch(g, vs, riemannian=True)[2],
                              batch=batch)
