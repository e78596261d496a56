"""Seeded synthetic inputs for the brickwall cost / gradient / HVP problem.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic, so both the CPU oracle and the GPU path can take
their inputs from it without sharing any computation.

Conventions (shared by every consumer of these arrays):

* Qubits are numbered q = 0 .. n-1.  A statevector index is
  x = sum_q b_q * 2**(n-1-q), i.e. qubit 0 is the most significant bit
  (Kronecker order).
* A brickwall of L layers: layer l (0-based, the first one applied to the
  input state) holds one two-qubit gate on every pair (q, q+1) with
  q = l (mod 2) and q + 1 < n (open boundary, Sec. III).  Gates are numbered
  layer by layer and, inside a layer, by increasing q.
* A gate is a complex 4x4 matrix G[i][j] with i the output and j the input
  index, i = 2*b_q + b_{q+1}.
* A product-state sample is n single-qubit states u_{s,q} = (amp of |0>,
  amp of |1>), drawn Haar-uniformly (normalised complex Gaussian vectors),
  as in the empirical risk of Sec. IV (Eq. costHS).
* Haar U(4) gates: QR of a complex Ginibre matrix with the phases of R's
  diagonal moved into Q (Mezzadri 2007).
* Directions V_k = G_k X_k with X_k anti-Hermitian, Gaussian, ||X_k||_F = 1,
  i.e. V lies in the tangent space of U(4)^K at G (App. F).
"""
from __future__ import annotations

import numpy as np


def num_gates(n: int, L: int) -> int:
    """Number of gates of an open-boundary brickwall with n qubits and L layers."""
    if n < 2 or L < 1:
        raise ValueError("need n >= 2 and L >= 1")
    return ((L + 1) // 2) * (n // 2) + (L // 2) * ((n - 1) // 2)


def gate_positions(n: int, L: int) -> list[tuple[int, int]]:
    """(layer, q) for every gate, in gate order."""
    out = []
    for layer in range(L):
        for q in range(layer % 2, n - 1, 2):
            out.append((layer, q))
    return out


def haar_unitary(rng: np.random.Generator, d: int, count: int) -> np.ndarray:
    """`count` Haar-random d x d unitaries, shape (count, d, d), complex128."""
    z = (rng.standard_normal((count, d, d)) + 1j * rng.standard_normal((count, d, d))) / np.sqrt(2.0)
    out = np.empty_like(z)
    for c in range(count):
        q, r = np.linalg.qr(z[c])
        ph = np.diagonal(r) / np.abs(np.diagonal(r))
        out[c] = q * ph[None, :]
    return out


def haar_qubit_states(rng: np.random.Generator, n_samples: int, n: int) -> np.ndarray:
    """Haar single-qubit states, shape (n_samples, n, 2), complex128, unit norm."""
    z = rng.standard_normal((n_samples, n, 2)) + 1j * rng.standard_normal((n_samples, n, 2))
    return z / np.linalg.norm(z, axis=-1, keepdims=True)


def random_antihermitian(rng: np.random.Generator, count: int) -> np.ndarray:
    """Gaussian anti-Hermitian 4x4 matrices with unit Frobenius norm, shape (count, 4, 4)."""
    a = rng.standard_normal((count, 4, 4)) + 1j * rng.standard_normal((count, 4, 4))
    x = 0.5 * (a - np.conj(np.swapaxes(a, -1, -2)))
    return x / np.linalg.norm(x, axis=(-1, -2), keepdims=True)


def random_tangent(rng: np.random.Generator, gates: np.ndarray) -> np.ndarray:
    """V_k = G_k X_k with X_k from `random_antihermitian`."""
    x = random_antihermitian(rng, gates.shape[0])
    return gates @ x


class Problem:
    """One synthetic problem instance (all arrays complex128, host memory)."""

    def __init__(self, n, L, L_ref, n_samples, G, V, uref, samples, seed):
        self.n, self.L, self.L_ref, self.n_samples = n, L, L_ref, n_samples
        self.G, self.V, self.uref, self.samples, self.seed = G, V, uref, samples, seed

    @property
    def K(self) -> int:
        return self.G.shape[0]


def make_problem(n: int, L: int, n_samples: int, seed: int, L_ref: int | None = None) -> Problem:
    """Haar brickwall G (depth L), Haar U_ref brickwall (depth L_ref, default 2L),
    Haar product samples and a random tangent direction V, from one seed."""
    if L_ref is None:
        L_ref = 2 * L
    rng = np.random.default_rng(seed)
    K = num_gates(n, L)
    K_ref = num_gates(n, L_ref)
    G = haar_unitary(rng, 4, K)
    uref = haar_unitary(rng, 4, K_ref)
    samples = haar_qubit_states(rng, n_samples, n)
    V = random_tangent(rng, G)
    return Problem(n, L, L_ref, n_samples, G, V, uref, samples, seed)


def to_interleaved(a: np.ndarray) -> np.ndarray:
    """complex128 array -> float64 array with a trailing (re, im) axis, C-contiguous."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64).reshape(a.shape + (2,))


def from_interleaved(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.view(np.complex128).reshape(a.shape[:-1])
