"""Translationally invariant brickwalls (App. E) on the device path.

* Per-layer gradient and HVP against the oracle (oracle/ti.py: expand, evaluate per gate, sum),
  both precisions, Euclidean and Riemannian, for an even n, an odd n (both layer kinds full) and
  n = 2, whose odd layers hold no gate (their derivatives are exactly zero); also with every pass
  boundary kept and with the boundaries rebuilt by the backward sweep.
* The device-side per-layer sums are exactly the sums, in increasing gate order, of the per-gate
  results of the same circuit expanded (bit for bit: the expansion copies the layer gates, and the
  per-gate evaluation is the one the per-gate calls run).
* Host and device-pointer TI calls give bitwise-equal results; invalid inputs found on the device
  leave every output untouched and set the device status.
"""
import numpy as np
import pytest

from oracle import riem, ti
from oracle.circuit import brickwall_positions
from parity import assert_close, assert_fidelity
from paper_2604_20384_amd.inputs import haar_unitary, make_problem, random_antihermitian

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}


def _ti_case(n, L, ns, seed):
    p = make_problem(n, L, ns, seed=seed)
    rng = np.random.default_rng(seed + 1)
    Gl = haar_unitary(rng, 4, L)
    Vl = Gl @ random_antihermitian(rng, L)
    return p, Gl, Vl


def _problem(p, precision, ckpt=1):
    from paper_2604_20384_amd.api import Problem
    return Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision=precision, ckpt_every=ckpt)


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


def _close_layers(got, ref, tol, what, n, L):
    """Layers holding gates meet the parity bar; layers without gates are exactly zero."""
    full = sorted({layer for layer, _ in brickwall_positions(n, L)})
    empty = [layer for layer in range(L) if layer not in full]
    assert all(np.all(got[layer] == 0) for layer in empty), (what, "empty layers not zero")
    return assert_close(got[full], ref[full], tol, what)


@pytest.mark.parametrize("n,L,ns", [(2, 4, 3), (7, 5, 3), (12, 6, 2)])
@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_ti_against_oracle(gpu, n, L, ns, precision):
    p, Gl, Vl = _ti_case(n, L, ns, 30 + n)
    tol = TOL[precision]
    ref = ti.evaluate(p.uref, p.samples, Gl, Vl, n, L, p.L_ref)
    gp = _problem(p, precision)
    c, g, h = gp.hvp_ti(Gl, Vl)
    assert_fidelity(gp.last_fidelity, ref["fidelity"], tol, (n, L, precision))
    _close_layers(g, ref["grad"], tol, "TI grad", n, L)
    _close_layers(h, ref["hvp"], tol, "TI hvp", n, L)
    c2, gR = gp.grad_ti(Gl, riemannian=True)
    _close_layers(gR, riem.riemannian_grad(Gl, ref["grad"]), tol, "TI Riemannian grad", n, L)
    c3, gR3, hR = gp.hvp_ti(Gl, Vl, riemannian=True)
    _close_layers(hR, riem.riemannian_hvp(Gl, ref["grad"], ref["hvp"], Vl), tol, "TI Riemannian hvp", n, L)
    gp.close()


@pytest.mark.parametrize("ckpt", [0, "rebuild"])
@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_ti_other_checkpoint_modes(gpu, precision, ckpt):
    """Every pass boundary kept, and the boundaries rebuilt by the backward sweep: same bars."""
    n, L = 11, 7
    p, Gl, Vl = _ti_case(n, L, 3, 71)
    tol = TOL[precision]
    ref = ti.evaluate(p.uref, p.samples, Gl, Vl, n, L, p.L_ref)
    gp = _problem(p, precision, ckpt)
    c, g, h = gp.hvp_ti(Gl, Vl)
    assert_fidelity(gp.last_fidelity, ref["fidelity"], tol, (precision, ckpt))
    _close_layers(g, ref["grad"], tol, ("TI grad", ckpt), n, L)
    _close_layers(h, ref["hvp"], tol, ("TI hvp", ckpt), n, L)
    gp.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("riemannian", [False, True])
def test_ti_sums_are_the_per_gate_sums(gpu, precision, riemannian):
    n, L = 9, 6
    p, Gl, Vl = _ti_case(n, L, 3, 44)
    gp = _problem(p, precision)
    c, g, h = gp.hvp(ti.expand(Gl, n, L), ti.expand(Vl, n, L), riemannian=riemannian)
    F = gp.last_fidelity
    ct, gt, ht = gp.hvp_ti(Gl, Vl, riemannian=riemannian)
    assert ct == c and gp.last_fidelity == F
    g_sum = np.zeros((L, 4, 4), dtype=np.complex128)
    h_sum = np.zeros((L, 4, 4), dtype=np.complex128)
    for k, (layer, _) in enumerate(brickwall_positions(n, L)):   # increasing gate order
        g_sum[layer] += g[k]
        h_sum[layer] += h[k]
    assert np.array_equal(gt, g_sum) and np.array_equal(ht, h_sum)
    gp.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("riemannian", [False, True])
def test_ti_dev_equals_host_bitwise(gpu, precision, riemannian):
    import torch
    n, L = 8, 5
    p, Gl, Vl = _ti_case(n, L, 4, 52)
    gp = _problem(p, precision)
    c, g, h = gp.hvp_ti(Gl, Vl, riemannian=riemannian)
    F = gp.last_fidelity
    cd, Fd, gd, hd = gp.hvp_ti_dev(_t(Gl), _t(Vl), riemannian=riemannian)
    c2, g2 = gp.grad_ti(Gl, riemannian=riemannian)
    c2d, F2d, g2d = gp.grad_ti_dev(_t(Gl), riemannian=riemannian)
    torch.cuda.synchronize()
    assert float(cd) == c and float(Fd) == F
    assert np.array_equal(gd.cpu().numpy(), g) and np.array_equal(hd.cpu().numpy(), h)
    assert float(c2d) == c2 and np.array_equal(g2d.cpu().numpy(), g2)
    assert gp.device_status() == 0
    gp.close()


def test_ti_dev_invalid_inputs_leave_outputs(gpu):
    import torch

    from paper_2604_20384_amd import _lib
    from paper_2604_20384_amd._lib import lib
    n, L = 6, 4
    p, Gl, Vl = _ti_case(n, L, 2, 61)
    gp = _problem(p, "c64")
    for bad, riemannian, status in (("nan", False, 1), ("nonunitary", True, 2)):
        G = Gl.copy()
        if bad == "nan":
            G[1, 2, 3] = np.nan
        else:
            G[2] = 1.5 * G[2]
        dG, dV = _t(G), _t(Vl)
        scal = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
        outs = [torch.full((L, 4, 4), 3 + 1j, dtype=torch.complex128, device="cuda") for _ in range(2)]
        st = lib.qhvp_hvp_ti_dev(gp.handle, dG.data_ptr(), dV.data_ptr(), int(riemannian), scal.data_ptr(),
                                 scal.data_ptr() + 8, outs[0].data_ptr(), outs[1].data_ptr())
        assert st == _lib.QHVP_OK, bad          # enqueued: the values are checked on the device
        assert gp.device_status() == status, bad
        torch.cuda.synchronize()
        assert bool(torch.all(scal == 7.0)), bad
        assert all(bool(torch.all(o == 3 + 1j)) for o in outs), bad
    # and the next valid call succeeds
    cd, Fd, gd, hd = gp.hvp_ti_dev(_t(Gl), _t(Vl))
    assert gp.device_status() == 0 and np.isfinite(float(cd))
    gp.close()
