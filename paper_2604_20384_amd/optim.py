"""Riemannian trust-region optimisation of brickwall gates on U(4)^K with a truncated conjugate-
gradient inner solver — the second-order method that consumes the HVP (Sec. IV: trust region with
truncated CG on the unitary manifold, after Absil, Mahony and Sepulchre, Alg. 10 and Alg. 11).

Metric: Re Tr(A^dag B) summed over gates.  Each inner CG iteration costs one Riemannian HVP; each
outer iteration one gradient (reused from the accepted point) and one cost evaluation.  The
retraction is the polar one of the library (the paper does not fix one).

`model` is any object with `cost(G) -> (cost, fidelity)`, `grad(G, riemannian=True) ->
(cost, grad)` and `hvp(G, V, riemannian=True) -> (cost, grad, hvp)`, e.g. `api.Problem`.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def inner(A: np.ndarray, B: np.ndarray) -> float:
    return float(np.real(np.vdot(A, B)))


def norm(A: np.ndarray) -> float:
    return float(np.sqrt(inner(A, A)))


@dataclasses.dataclass
class TCGResult:
    eta: np.ndarray
    Heta: np.ndarray
    iterations: int
    stop: str


def truncated_cg(model, G, grad, radius, theta=1.0, kappa=0.1, max_iter=None) -> TCGResult:
    """Steihaug-Toint truncated CG for min <grad, eta> + 1/2 <eta, H eta>, |eta| <= radius."""
    K = G.shape[0]
    max_iter = 16 * K if max_iter is None else max_iter
    eta = np.zeros_like(grad)
    Heta = np.zeros_like(grad)
    r = grad.copy()
    r0 = norm(r)
    rr = inner(r, r)
    delta = -r
    for j in range(max_iter):
        Hd = model.hvp(G, delta, riemannian=True)[2]
        dHd = inner(delta, Hd)
        if dHd <= 0:                                         # negative curvature: go to the boundary
            tau = _to_boundary(eta, delta, radius)
            return TCGResult(eta + tau * delta, Heta + tau * Hd, j + 1, "negative curvature")
        alpha = rr / dHd
        eta_new = eta + alpha * delta
        if norm(eta_new) >= radius:                          # step leaves the trust region
            tau = _to_boundary(eta, delta, radius)
            return TCGResult(eta + tau * delta, Heta + tau * Hd, j + 1, "trust-region boundary")
        eta, Heta = eta_new, Heta + alpha * Hd
        r = r + alpha * Hd
        rr_new = inner(r, r)
        if np.sqrt(rr_new) <= r0 * min(r0 ** theta, kappa):
            return TCGResult(eta, Heta, j + 1, "residual")
        delta = -r + (rr_new / rr) * delta
        rr = rr_new
    return TCGResult(eta, Heta, max_iter, "max iterations")


def _to_boundary(eta, delta, radius):
    """tau >= 0 with |eta + tau delta| = radius."""
    a = inner(delta, delta)
    b = 2 * inner(eta, delta)
    c = inner(eta, eta) - radius ** 2
    return (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)


@dataclasses.dataclass
class TRHistory:
    cost: list
    grad_norm: list
    radius: list
    accepted: list
    inner_iterations: list
    hvp_calls: int = 0


def trust_region(model, G0, retract, radius=0.5, max_radius=None, rho_accept=0.1, max_iter=50,
                 grad_tol=1e-9, tcg_kwargs=None):
    """Riemannian trust region (accept if rho > rho_accept; shrink by 4 if rho < 1/4, grow by 2 if
    rho > 3/4 at the boundary).  `retract(G, xi)` maps a tangent step to U(4)^K."""
    tcg_kwargs = tcg_kwargs or {}
    max_radius = 8 * radius if max_radius is None else max_radius
    G = np.array(G0, dtype=np.complex128)
    f, g = model.grad(G, riemannian=True)
    hist = TRHistory([f], [norm(g)], [radius], [], [])
    for _ in range(max_iter):
        if norm(g) <= grad_tol:
            break
        res = truncated_cg(model, G, g, radius, **tcg_kwargs)
        hist.hvp_calls += res.iterations
        model_decrease = -(inner(g, res.eta) + 0.5 * inner(res.eta, res.Heta))
        if model_decrease <= 1e-14 * max(1.0, abs(f)):
            break          # the model predicts no decrease the cost (1 - F in FP64) could resolve
        G_new = retract(G, res.eta)
        f_new, _ = model.cost(G_new)
        rho = (f - f_new) / model_decrease if model_decrease > 0 else -np.inf
        at_boundary = abs(norm(res.eta) - radius) <= 1e-9 * radius
        if rho < 0.25:
            radius = radius / 4
        elif rho > 0.75 and at_boundary:
            radius = min(2 * radius, max_radius)
        accepted = rho > rho_accept
        if accepted:
            G = G_new
            f, g = model.grad(G, riemannian=True)
        hist.cost.append(f)
        hist.grad_norm.append(norm(g))
        hist.radius.append(radius)
        hist.accepted.append(bool(accepted))
        hist.inner_iterations.append(res.iterations)
    return G, hist
