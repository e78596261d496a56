"""The HVP entry point that allocates nothing (qhvp_hvp_noalloc), through the C ABI.

It must match the device-pointer HVP it is a variant of (qhvp_hvp_dev on a problem created for the
same inputs) to the parity bar (complex64 1e-5, complex128 1e-10), on two calls in a row with the
second smaller than the first.  It shares the kernels and their order of arithmetic, so the results
are in fact equal bit for bit, which is checked too.  It must refuse a problem beyond its scratch
with QHVP_ERR_NOMEM before enqueueing anything, and the device's free memory must not change across
its calls.
"""
import numpy as np
import pytest

from parity import assert_close, assert_fidelity
from paper_2604_20384_amd.inputs import make_problem

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}
PREC = {"c128": 0, "c64": 1}


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


class _Call:
    """Device inputs and outputs of one noalloc call, allocated before the call."""

    def __init__(self, p):
        import torch
        self.p = p
        self.uref, self.samples, self.G, self.V = _t(p.uref), _t(p.samples), _t(p.G), _t(p.V)
        K = p.G.shape[0]
        self.scal = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        self.g = torch.empty((K, 4, 4), dtype=torch.complex128, device="cuda")
        self.h = torch.empty((K, 4, 4), dtype=torch.complex128, device="cuda")

    def run(self, ctx, precision):
        import torch

        from paper_2604_20384_amd._lib import lib
        p = self.p
        return lib.qhvp_hvp_noalloc(ctx.handle, p.n, p.L, p.L_ref, self.uref.data_ptr(), self.samples.data_ptr(),
                                    p.n_samples, PREC[precision], self.G.data_ptr(), self.V.data_ptr(), 0,
                                    self.scal.data_ptr(), self.scal.data_ptr() + 8, self.g.data_ptr(),
                                    self.h.data_ptr(), torch.cuda.current_stream().cuda_stream)


def _reference(p, precision):
    from paper_2604_20384_amd.api import Problem
    gp = Problem(p.n, p.L, p.uref, p.samples, L_ref=p.L_ref, precision=precision, ckpt_every=0)
    c, F, g, h = gp.hvp_dev(_t(p.G), _t(p.V))
    out = (float(c), float(F), g.cpu().numpy(), h.cpu().numpy())
    gp.close()
    return out


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_noalloc_matches_hvp_dev_on_two_calls(gpu, precision):
    import torch

    from paper_2604_20384_amd import _lib
    from paper_2604_20384_amd.api import default_context
    ctx = default_context(0)
    problems = [make_problem(12, 6, 16, seed=81), make_problem(9, 4, 5, seed=82)]   # the second is smaller
    calls = [_Call(p) for p in problems]
    got = []
    for i, call in enumerate(calls):
        st = call.run(ctx, precision)
        assert st == _lib.QHVP_OK, _lib.lib.qhvp_last_error().decode()
        torch.cuda.synchronize()
        got.append((float(call.scal[0]), float(call.scal[1]), call.g.cpu().numpy(), call.h.cpu().numpy()))
        if i == 0:
            # the first launches of a process set up the runtime's own state; from here on the
            # calls must not change the device's free memory
            free0 = torch.cuda.mem_get_info()[0]
    for call in calls:
        assert call.run(ctx, precision) == _lib.QHVP_OK
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    for p, (c, F, g, h) in zip(problems, got):
        rc, rF, rg, rh = _reference(p, precision)
        assert_fidelity(F, rF, TOL[precision], "noalloc fidelity")
        assert abs(c - rc) <= TOL[precision]
        assert_close(g, rg, TOL[precision], "noalloc grad")
        assert_close(h, rh, TOL[precision], "noalloc hvp")
        assert c == rc and F == rF and np.array_equal(g, rg) and np.array_equal(h, rh)


def test_noalloc_refuses_problems_beyond_its_scratch(gpu):
    import torch

    from paper_2604_20384_amd import _lib
    from paper_2604_20384_amd.api import default_context
    ctx = default_context(0)
    call = _Call(make_problem(20, 20, 256, seed=83))     # ~2 GiB per state set: far beyond 64 MiB
    st = call.run(ctx, "c64")
    assert st == _lib.QHVP_ERR_NOMEM
    assert "MiB of scratch" in _lib.lib.qhvp_last_error().decode()
    torch.cuda.synchronize()
    assert bool(torch.isnan(call.scal).all())            # nothing was enqueued
