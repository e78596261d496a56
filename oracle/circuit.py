"""Brickwall circuits on full statevectors (oracle; test infrastructure only).

Layout (Sec. III "Problem setting"; the figure that draws it is missing, so
the reading is: open boundary, first layer on the pairs (0,1), (2,3), ...,
second on (1,2), (3,4), ..., alternating).  Gate k acts as
I_{2^q} (x) G_k (x) I_{2^{n-q-2}} on qubits (q, q+1), qubit 0 being the most
significant bit of the statevector index.
"""
from __future__ import annotations

import numpy as np


def brickwall_positions(n: int, L: int) -> list[tuple[int, int]]:
    """(layer, q) of each gate in application order."""
    pos = []
    for layer in range(L):
        start = layer % 2
        q = start
        while q + 1 < n:
            pos.append((layer, q))
            q += 2
    return pos


def product_state(u: np.ndarray) -> np.ndarray:
    """psi = u_0 (x) u_1 (x) ... (x) u_{n-1} for u of shape (n, 2) (Sec. IV, Haar product states)."""
    psi = np.ones(1, dtype=np.complex128)
    for q in range(u.shape[0]):
        psi = np.kron(psi, u[q])
    return psi


def embed(G: np.ndarray, q: int, n: int) -> np.ndarray:
    """Dense 2^n x 2^n operator I (x) G (x) I with G on qubits (q, q+1)."""
    return np.kron(np.kron(np.eye(2 ** q), G), np.eye(2 ** (n - q - 2)))


def dense_circuit(gates: np.ndarray, n: int, L: int) -> np.ndarray:
    """The composed map G_K ... G_1 as a dense matrix (Sec. II.B, the composition of linear maps)."""
    pos = brickwall_positions(n, L)
    assert len(pos) == gates.shape[0]
    U = np.eye(2 ** n, dtype=np.complex128)
    for k, (_, q) in enumerate(pos):
        U = embed(gates[k], q, n) @ U
    return U


def apply_gate(state: np.ndarray, G: np.ndarray, q: int, n: int) -> np.ndarray:
    """Apply the 4x4 matrix G on qubits (q, q+1) of a batch of statevectors.

    `state` has shape (2^n, ...) (extra trailing axes are batch axes).
    """
    batch = state.shape[1:]
    t = state.reshape((2 ** q, 4, 2 ** (n - q - 2)) + batch)
    t = np.tensordot(G, t, axes=([1], [1]))          # (4, 2^q, 2^(n-q-2), batch)
    t = np.moveaxis(t, 0, 1)
    return t.reshape((2 ** n,) + batch)


def apply_circuit(state: np.ndarray, gates: np.ndarray, n: int, L: int) -> np.ndarray:
    for k, (_, q) in enumerate(brickwall_positions(n, L)):
        state = apply_gate(state, gates[k], q, n)
    return state


def pair_unfold(state: np.ndarray, q: int, n: int) -> np.ndarray:
    """Reshape a statevector to (4, 2^(n-2)): pair index (b_q, b_{q+1}) first, the rest (alpha) second."""
    t = state.reshape(2 ** q, 4, 2 ** (n - q - 2))
    return np.moveaxis(t, 1, 0).reshape(4, -1)


def labels(uref: np.ndarray, samples: np.ndarray, n: int, L_ref: int) -> tuple[np.ndarray, np.ndarray]:
    """psi_s and phi_s = U_ref psi_s for all samples (Sec. III, Eq. costHS); arrays (N_s, 2^n)."""
    psi = np.stack([product_state(samples[s]) for s in range(samples.shape[0])])
    phi = apply_circuit(psi.T.copy(), uref, n, L_ref).T.copy()
    return psi, phi
