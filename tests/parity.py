"""Parity bars shared by the GPU tests (HIP path against the CPU oracle).

Floating-point bars (written in each test): complex128 1e-10, complex64 with FP64 accumulation 1e-5,
relative.  A result over K gates (K x 4 x 4 complex) must meet the bar twice: globally,
||got - ref||_2 / ||ref||_2, and gate by gate, max_ij |got_k - ref_k| / max_ij |ref_k| for every k, so
that an error confined to gates with small entries cannot hide in the global norm.  The fidelity
F = mean_s |T_s|^2 is compared relatively (the cost C = 1 - F is ~1 and a relative error on it is
vacuous).
"""
import numpy as np


def rel(got, ref) -> float:
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def per_gate_rel(got, ref) -> float:
    """Largest over gates k of max_ij |got_k - ref_k| / max_ij |ref_k|."""
    got = np.asarray(got).reshape(-1, 16)
    ref = np.asarray(ref).reshape(-1, 16)
    num = np.max(np.abs(got - ref), axis=1)
    den = np.max(np.abs(ref), axis=1)
    return float(np.max(num / den))


def assert_close(got, ref, tol, what=""):
    g, k = rel(got, ref), per_gate_rel(got, ref)
    assert g <= tol and k <= tol, (what, "global", g, "per gate", k, "tol", tol)
    return g, k


def assert_fidelity(F, F_ref, tol, what=""):
    e = abs(F - F_ref) / F_ref
    assert e <= tol, (what, "fidelity", F, F_ref, e)
    return e
