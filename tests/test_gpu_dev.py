"""The device-pointer calls (*_dev) of the C ABI on torch tensors.

* Host and device calls run the same device code, so their results are equal bit for bit
  (complex128 and complex64, Euclidean and Riemannian, one-shot and two-phase).
* Outputs are left untouched on every error path: host-side argument errors (both call kinds),
  and values the device rejects (non-finite G or V, non-unitary G in Riemannian mode), which the
  device-side status reports.
* A host pointer passed where device memory is expected is refused before anything is enqueued.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import circuit, sv
from parity import assert_close, assert_fidelity
from paper_2604_20384_amd.inputs import make_problem

pytestmark = pytest.mark.gpu


def _problem(p, precision, with_tangent=True):
    from paper_2604_20384_amd.api import Problem
    return Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision=precision, ckpt_every=1,
                   with_tangent=with_tangent)


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("riemannian", [False, True])
def test_dev_calls_equal_host_calls_bitwise(gpu, precision, riemannian):
    import torch
    p = make_problem(11, 5, 6, seed=71)
    gp = _problem(p, precision)
    c, g, h = gp.hvp(p.G, p.V, riemannian=riemannian)
    F = gp.last_fidelity
    cd, Fd, gd, hd = gp.hvp_dev(_t(p.G), _t(p.V), riemannian=riemannian)
    torch.cuda.synchronize()
    assert float(cd) == c and float(Fd) == F
    assert np.array_equal(gd.cpu().numpy(), g) and np.array_equal(hd.cpu().numpy(), h)
    c2, g2 = gp.grad(p.G, riemannian=riemannian)
    c2d, F2d, g2d = gp.grad_dev(_t(p.G), riemannian=riemannian)
    assert float(c2d) == c2 and np.array_equal(g2d.cpu().numpy(), g2)
    c3, F3 = gp.cost(p.G)
    c3d, F3d = gp.cost_dev(_t(p.G))
    assert float(c3d) == c3 and float(F3d) == F3
    # two-phase form
    c4d, F4d = gp.forward_dev(_t(p.G), _t(p.V), riemannian=riemannian)
    g4d, h4d = gp.backward_dev()
    assert float(c4d) == c and np.array_equal(g4d.cpu().numpy(), g) and np.array_equal(h4d.cpu().numpy(), h)
    # and against the oracle
    if not riemannian:
        psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
        ref = sv.evaluate(psi, phi, p.G, p.V, p.n, p.L)
        tol = {"c128": 1e-10, "c64": 1e-5}[precision]
        assert_fidelity(float(Fd), ref["fidelity"], tol, "dev")
        assert_close(gd.cpu().numpy(), ref["grad"], tol, "dev grad")
        assert_close(hd.cpu().numpy(), ref["hvp"], tol, "dev hvp")
    gp.close()


def test_dev_recompute_backward(gpu, monkeypatch):
    """The device-side choice of the backward algorithm follows QHVP_BACKWARD on the dev path too."""
    import torch
    p = make_problem(12, 5, 3, seed=72)
    gp = _problem(p, "c64")
    _, _, g_i, h_i = gp.hvp_dev(_t(p.G), _t(p.V))
    torch.cuda.synchronize()
    assert gp.backward_from_outputs
    monkeypatch.setenv("QHVP_BACKWARD", "recompute")
    _, _, g_r, h_r = gp.hvp_dev(_t(p.G), _t(p.V))
    torch.cuda.synchronize()
    assert not gp.backward_from_outputs
    assert_close(g_i.cpu().numpy(), g_r.cpu().numpy(), 1e-5, "grad")
    assert_close(h_i.cpu().numpy(), h_r.cpu().numpy(), 1e-5, "hvp")
    gp.close()


def _sentinel(shape):
    return np.full(shape, 7.25, dtype=np.float64)


def test_host_call_errors_leave_outputs_untouched(gpu):
    from paper_2604_20384_amd import _lib
    from paper_2604_20384_amd._lib import dptr, lib
    p = make_problem(8, 4, 3, seed=73)
    gp = _problem(p, "c128")
    K = gp.K
    Gf = np.ascontiguousarray(p.G).view(np.float64).copy()
    Vf = np.ascontiguousarray(p.V).view(np.float64).copy()
    cases = []
    Gnan = Gf.copy()
    Gnan[5] = np.nan
    cases.append(("nan G", Gnan, Vf, 0, _lib.QHVP_ERR_INVALID))
    Vinf = Vf.copy()
    Vinf[0] = np.inf
    cases.append(("inf V", Gf, Vinf, 0, _lib.QHVP_ERR_INVALID))
    cases.append(("non-unitary Riemannian", Gf + 0.1, Vf, 1, _lib.QHVP_ERR_INVALID))
    for what, G, V, geom, want in cases:
        cost, fid = _sentinel(1), _sentinel(1)
        grad, hvp = _sentinel(K * 32), _sentinel(K * 32)
        st = lib.qhvp_hvp(gp.handle, dptr(G), dptr(V), geom, dptr(cost), dptr(fid), dptr(grad), dptr(hvp))
        assert st == want, what
        for o in (cost, fid, grad, hvp):
            assert np.all(o == 7.25), what
    # a problem without tangent storage refuses an HVP before anything runs
    gq = _problem(p, "c128", with_tangent=False)
    cost, grad, hvp = _sentinel(1), _sentinel(K * 32), _sentinel(K * 32)
    st = lib.qhvp_hvp(gq.handle, dptr(Gf), dptr(Vf), 0, dptr(cost), None, dptr(grad), dptr(hvp))
    assert st == _lib.QHVP_ERR_UNSUPPORTED
    assert np.all(cost == 7.25) and np.all(grad == 7.25) and np.all(hvp == 7.25)
    gq.close()
    gp.close()


def test_dev_errors_leave_outputs_untouched(gpu):
    import torch

    from paper_2604_20384_amd import _lib
    from paper_2604_20384_amd._lib import lib
    p = make_problem(8, 4, 3, seed=74)
    gp = _problem(p, "c64")
    K = gp.K

    def outs():
        return (torch.full((2,), 7.25, dtype=torch.float64, device="cuda"),
                torch.full((K, 4, 4, 2), 7.25, dtype=torch.float64, device="cuda"),
                torch.full((K, 4, 4, 2), 7.25, dtype=torch.float64, device="cuda"))

    G, V = _t(p.G), _t(p.V)
    Gnan = G.clone()
    Gnan[3, 1, 2] = complex(float("nan"), 0.0)
    for what, Gi, Vi, geom, status in (("nan G", Gnan, V, 0, 1), ("non-unitary Riemannian", G + 0.1, V, 1, 2)):
        s, g, h = outs()
        st = lib.qhvp_hvp_dev(gp.handle, Gi.data_ptr(), Vi.data_ptr(), geom, s.data_ptr(), s.data_ptr() + 8,
                              g.data_ptr(), h.data_ptr())
        assert st == _lib.QHVP_OK, what          # enqueued: the values are checked on the device
        assert gp.device_status() == status, what
        torch.cuda.synchronize()
        for o in (s, g, h):
            assert bool(torch.all(o == 7.25)), what
    # a valid call afterwards runs normally and clears the status
    s, g, h = outs()
    st = lib.qhvp_hvp_dev(gp.handle, G.data_ptr(), V.data_ptr(), 0, s.data_ptr(), s.data_ptr() + 8, g.data_ptr(),
                          h.data_ptr())
    assert st == _lib.QHVP_OK and gp.device_status() == 0
    torch.cuda.synchronize()
    assert not bool(torch.any(g == 7.25))
    # host memory where device memory is expected: refused on the host, nothing enqueued
    Gh = np.ascontiguousarray(p.G).view(np.float64).copy()
    s, g, h = outs()
    st = lib.qhvp_hvp_dev(gp.handle, Gh.ctypes.data, V.data_ptr(), 0, s.data_ptr(), s.data_ptr() + 8,
                          g.data_ptr(), h.data_ptr())
    assert st == _lib.QHVP_ERR_INVALID
    assert "device memory" in lib.qhvp_last_error().decode()
    torch.cuda.synchronize()
    assert bool(torch.all(g == 7.25))
    # no direction on a dev HVP, and a backward without a forward
    assert lib.qhvp_hvp_dev(gp.handle, G.data_ptr(), None, 0, None, None, None, h.data_ptr()) == _lib.QHVP_ERR_INVALID
    gp.hvp_dev(G, V)
    assert lib.qhvp_backward_dev(gp.handle, g.data_ptr(), None) == _lib.QHVP_ERR_INVALID
    gp.close()
