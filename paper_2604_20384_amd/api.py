"""Python binding of the qhvp C ABI: `Context` and `Problem`.

Device memory for the workspace comes from PyTorch (so its peak HBM is
visible to `torch.cuda.max_memory_allocated`), and the HIP stream is a torch
stream; everything else is marshalling.  Host calls take and return numpy
complex128 arrays of shape (K, 4, 4); the *_dev calls take and return torch
complex128 tensors on the problem's device and run asynchronously on the
problem's stream (no host copy of G, V or the results).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import check, dptr, lib

PRECISIONS = {"c128": _lib.QHVP_C128, "c64": _lib.QHVP_C64_ACC64}
CKPT_REBUILD = _lib.QHVP_CKPT_REBUILD


def num_gates(n: int, L: int) -> int:
    return lib.qhvp_num_gates(n, L)


def plan(n: int, L: int):
    """The library's pass plan: (gates per pass, gate indices in application order)."""
    K = num_gates(n, L)
    np_ = lib.qhvp_plan(n, L, 0, None, None)
    if np_ < 0:
        check(-np_)
    per = (C.c_int * np_)()
    order = (C.c_int * K)()
    got = lib.qhvp_plan(n, L, np_, per, order)
    if got < 0:
        check(-got)
    return list(per), list(order)


def _ckpt(ckpt_every) -> int:
    """The library's checkpoint setting: an int, or "rebuild" (QHVP_CKPT_REBUILD)."""
    return CKPT_REBUILD if ckpt_every == "rebuild" else int(ckpt_every)


def workspace_bytes(n, L, L_ref, n_samples, precision="c128", ckpt_every=1, with_tangent=True) -> int:
    return int(lib.qhvp_workspace_bytes(n, L, L_ref, n_samples, PRECISIONS[precision], _ckpt(ckpt_every),
                                        1 if with_tangent else 0))


def _c128(a, shape=None) -> np.ndarray:
    if hasattr(a, "detach"):          # torch tensor
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _f64(a: np.ndarray) -> np.ndarray:
    return a.view(np.float64)


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib.qhvp_ctx_create(device, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib.qhvp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


class Problem:
    """One (U_ref, samples) problem on the device; cost / grad / hvp for any gates G.

    n, L        : qubits and ansatz layers (K = num_gates(n, L) gates).
    uref        : (K_ref, 4, 4) gates of the reference brickwall of L_ref layers.
    samples     : (N_s, n, 2) single-qubit states of the product-state samples.
    precision   : "c128" or "c64" (complex64 states, FP64 accumulation).
    ckpt_every  : layer-checkpoint interval (0 = keep every pass boundary, c > 0 every c layers,
                  -c every c passes), or "rebuild": keep only the final forward states and let the
                  backward sweep rebuild the pass boundaries (well-conditioned gates).
    workspace   : "torch" (allocate with torch), a (device pointer, bytes) block owned by the
                  caller, or None (the library allocates).
    """

    def __init__(self, n, L, uref, samples, L_ref=None, precision="c128", ckpt_every=1,
                 with_tangent=True, device=0, stream=None, workspace="torch"):
        import torch

        self.n, self.L = int(n), int(L)
        self.K = num_gates(n, L)
        uref = _c128(uref)
        if L_ref is None:
            L_ref = self._layers_of(uref.shape[0])
        self.L_ref = int(L_ref)
        self.K_ref = num_gates(n, L_ref)
        uref = _c128(uref, (self.K_ref, 4, 4))
        samples = _c128(samples)
        if samples.ndim != 3 or samples.shape[1:] != (n, 2):
            raise ValueError(f"samples must have shape (N_s, {n}, 2)")
        self.n_samples = samples.shape[0]
        self.precision = precision
        self.ctx = default_context(device)
        self.device = device
        self.ws_bytes = workspace_bytes(n, L, L_ref, self.n_samples, precision, ckpt_every, with_tangent)
        if self.ws_bytes == 0:
            raise ValueError("invalid problem shape")
        self._ws = None
        ws_ptr = None
        if isinstance(workspace, str) and workspace == "torch":
            self._ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=f"cuda:{device}")
            ws_ptr = C.c_void_p(self._ws.data_ptr())
        elif isinstance(workspace, tuple):           # (device pointer, bytes) owned by the caller
            if workspace[1] < self.ws_bytes:
                raise MemoryError(f"workspace block of {workspace[1]} bytes, need {self.ws_bytes}")
            ws_ptr = C.c_void_p(int(workspace[0]))
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        check(lib.qhvp_problem_create(self.ctx.handle, n, L, L_ref, dptr(_f64(uref)), dptr(_f64(samples)),
                                      self.n_samples, PRECISIONS[precision], _ckpt(ckpt_every),
                                      1 if with_tangent else 0, ws_ptr, self.ws_bytes,
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self.epoch = 0          # bumped by every device evaluation (checkpoints are overwritten)

    def _layers_of(self, K_ref):
        for Lr in range(1, 10000):
            if num_gates(self.n, Lr) == K_ref:
                return Lr
        raise ValueError("cannot infer L_ref from the number of U_ref gates")

    # ------------------------------------------------------------------
    def cost(self, G):
        self.epoch += 1
        G = _c128(G, (self.K, 4, 4))
        c, f = C.c_double(), C.c_double()
        check(lib.qhvp_cost(self.handle, dptr(_f64(G)), C.byref(c), C.byref(f)))
        self.last_fidelity = f.value
        return c.value, f.value

    def grad(self, G, riemannian=False):
        """(cost, gradient); the fidelity F of the call (as computed, not 1 - cost) is in
        `last_fidelity`."""
        self.epoch += 1
        G = _c128(G, (self.K, 4, 4))
        g = np.empty((self.K, 4, 4), dtype=np.complex128)
        c, f = C.c_double(), C.c_double()
        check(lib.qhvp_grad(self.handle, dptr(_f64(G)), int(riemannian), C.byref(c), C.byref(f), dptr(_f64(g))))
        self.last_fidelity = f.value
        return c.value, g

    def hvp(self, G, V, riemannian=False):
        """(cost, gradient, HVP along V); the call's fidelity is in `last_fidelity`."""
        self.epoch += 1
        G = _c128(G, (self.K, 4, 4))
        V = _c128(V, (self.K, 4, 4))
        g = np.empty((self.K, 4, 4), dtype=np.complex128)
        h = np.empty((self.K, 4, 4), dtype=np.complex128)
        c, f = C.c_double(), C.c_double()
        check(lib.qhvp_hvp(self.handle, dptr(_f64(G)), dptr(_f64(V)), int(riemannian), C.byref(c), C.byref(f),
                           dptr(_f64(g)), dptr(_f64(h))))
        self.last_fidelity = f.value
        return c.value, g, h

    # ---- device-pointer calls on torch tensors (complex128, shape (K, 4, 4), on the problem's device)
    def _dev_in(self, t, name, count=None):
        import torch
        count = self.K if count is None else count
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or t.shape != (count, 4, 4):
            raise ValueError(f"{name} must be a complex128 torch tensor of shape ({count}, 4, 4)")
        if t.device != torch.device(f"cuda:{self.device}"):
            raise ValueError(f"{name} must be on cuda:{self.device}")
        return t.contiguous()

    def _dev_out(self, n_mats, count=None):
        import torch
        dev = f"cuda:{self.device}"
        count = self.K if count is None else count
        scal = torch.empty(2, dtype=torch.float64, device=dev)
        mats = [torch.empty((count, 4, 4), dtype=torch.complex128, device=dev) for _ in range(n_mats)]
        return scal, mats

    def cost_dev(self, G):
        """(cost, fidelity) as 0-dim float64 device tensors, enqueued on the problem's stream."""
        self.epoch += 1
        G = self._dev_in(G, "G")
        scal, _ = self._dev_out(0)
        check(lib.qhvp_cost_dev(self.handle, G.data_ptr(), scal.data_ptr(), scal.data_ptr() + 8))
        self._dev_keep = (G,)   # alive until the enqueued work has read it
        return scal[0], scal[1]

    def grad_dev(self, G, riemannian=False):
        """(cost, fidelity, gradient) as device tensors; G never leaves the device."""
        self.epoch += 1
        G = self._dev_in(G, "G")
        scal, (g,) = self._dev_out(1)
        check(lib.qhvp_grad_dev(self.handle, G.data_ptr(), int(riemannian), scal.data_ptr(), scal.data_ptr() + 8,
                                g.data_ptr()))
        self._dev_keep = (G,)
        return scal[0], scal[1], g

    def hvp_dev(self, G, V, riemannian=False):
        """(cost, fidelity, gradient, HVP along V) as device tensors."""
        self.epoch += 1
        G, V = self._dev_in(G, "G"), self._dev_in(V, "V")
        scal, (g, h) = self._dev_out(2)
        check(lib.qhvp_hvp_dev(self.handle, G.data_ptr(), V.data_ptr(), int(riemannian), scal.data_ptr(),
                               scal.data_ptr() + 8, g.data_ptr(), h.data_ptr()))
        self._dev_keep = (G, V)
        return scal[0], scal[1], g, h

    def forward_dev(self, G, V=None, riemannian=False):
        """Forward sweep on device tensors (keeps the checkpoints for one `backward_dev`);
        returns (cost, fidelity) as device tensors."""
        self.epoch += 1
        G = self._dev_in(G, "G")
        Vd = None if V is None else self._dev_in(V, "V")
        scal, _ = self._dev_out(0)
        check(lib.qhvp_forward_dev(self.handle, G.data_ptr(), None if Vd is None else Vd.data_ptr(),
                                   int(riemannian), scal.data_ptr(), scal.data_ptr() + 8))
        self._fwd_tangent = V is not None
        self._dev_keep = (G, Vd)   # the inputs stay alive until the enqueued sweep has read them
        return scal[0], scal[1]

    def backward_dev(self):
        """Backward sweep of the last `forward_dev`: grad, or (grad, hvp), as device tensors."""
        self.epoch += 1
        tang = getattr(self, "_fwd_tangent", False)
        _, mats = self._dev_out(2 if tang else 1)
        check(lib.qhvp_backward_dev(self.handle, mats[0].data_ptr(), mats[1].data_ptr() if tang else None))
        return mats[0] if not tang else (mats[0], mats[1])

    def device_status(self) -> int:
        """Device-side input check of the last call (waits for the stream): 0 if valid."""
        st = C.c_int()
        check(lib.qhvp_device_status(self.handle, C.byref(st)))
        return st.value

    def hvp_batch(self, G, Vs, riemannian=False):
        """HVPs at one G along several directions Vs (M, K, 4, 4) -> (cost, grad, (M, K, 4, 4)).

        Equal bit for bit to M calls of `hvp`; the forward states at G are stored by the first
        direction (or kept from an earlier gradient / HVP call at the same G) and read by the rest."""
        self.epoch += 1
        G = _c128(G, (self.K, 4, 4))
        Vs = _c128(Vs)
        if Vs.ndim != 4 or Vs.shape[1:] != (self.K, 4, 4) or Vs.shape[0] < 1:
            raise ValueError(f"Vs must have shape (M, {self.K}, 4, 4) with M >= 1")
        M = Vs.shape[0]
        g = np.empty((self.K, 4, 4), dtype=np.complex128)
        h = np.empty((M, self.K, 4, 4), dtype=np.complex128)
        c = C.c_double()
        check(lib.qhvp_hvp_batch(self.handle, dptr(_f64(G)), M, dptr(_f64(Vs)), int(riemannian), C.byref(c),
                                 dptr(_f64(g)), dptr(_f64(h))))
        return c.value, g, h

    def states_kept_for(self, G) -> bool:
        """Whether the forward states kept at the pass boundaries belong to gates G (bitwise)."""
        G = _c128(G, (self.K, 4, 4))
        r = lib.qhvp_states_kept_for(self.handle, dptr(_f64(G)))
        if r < 0:
            raise ValueError("closed problem")
        return bool(r)

    def forward(self, G, V=None, riemannian=False):
        """Forward sweep (keeps the checkpoints for one `backward`); returns (cost, fidelity)."""
        self.epoch += 1
        G = _c128(G, (self.K, 4, 4))
        Vp = None if V is None else dptr(_f64(_c128(V, (self.K, 4, 4))))
        c, f = C.c_double(), C.c_double()
        check(lib.qhvp_forward(self.handle, dptr(_f64(G)), Vp, int(riemannian), C.byref(c), C.byref(f)))
        self._fwd_tangent = V is not None
        self.last_fidelity = f.value
        return c.value, f.value

    def backward(self):
        """Backward sweep of the last `forward`; returns grad, or (grad, hvp) after a forward with V."""
        self.epoch += 1
        g = np.empty((self.K, 4, 4), dtype=np.complex128)
        h = np.empty((self.K, 4, 4), dtype=np.complex128) if getattr(self, "_fwd_tangent", False) else None
        check(lib.qhvp_backward(self.handle, dptr(_f64(g)), None if h is None else dptr(_f64(h))))
        return g if h is None else (g, h)

    # ---- translationally invariant circuits (App. E): one (4, 4) gate per layer, shape (L, 4, 4)
    def grad_ti(self, G_layers, riemannian=False):
        self.epoch += 1
        G = _c128(G_layers, (self.L, 4, 4))
        g = np.empty((self.L, 4, 4), dtype=np.complex128)
        c, f = C.c_double(), C.c_double()
        check(lib.qhvp_grad_ti(self.handle, dptr(_f64(G)), int(riemannian), C.byref(c), C.byref(f), dptr(_f64(g))))
        self.last_fidelity = f.value
        return c.value, g

    def hvp_ti(self, G_layers, V_layers, riemannian=False):
        self.epoch += 1
        G = _c128(G_layers, (self.L, 4, 4))
        V = _c128(V_layers, (self.L, 4, 4))
        g = np.empty((self.L, 4, 4), dtype=np.complex128)
        h = np.empty((self.L, 4, 4), dtype=np.complex128)
        c, f = C.c_double(), C.c_double()
        check(lib.qhvp_hvp_ti(self.handle, dptr(_f64(G)), dptr(_f64(V)), int(riemannian), C.byref(c), C.byref(f),
                              dptr(_f64(g)), dptr(_f64(h))))
        self.last_fidelity = f.value
        return c.value, g, h

    def grad_ti_dev(self, G_layers, riemannian=False):
        """(cost, fidelity, per-layer gradient) as device tensors; G_layers (L, 4, 4) on the device."""
        self.epoch += 1
        G = self._dev_in(G_layers, "G_layers", self.L)
        scal, (g,) = self._dev_out(1, self.L)
        check(lib.qhvp_grad_ti_dev(self.handle, G.data_ptr(), int(riemannian), scal.data_ptr(), scal.data_ptr() + 8,
                                   g.data_ptr()))
        self._dev_keep = (G,)
        return scal[0], scal[1], g

    def hvp_ti_dev(self, G_layers, V_layers, riemannian=False):
        """(cost, fidelity, per-layer gradient, per-layer HVP along V_layers) as device tensors."""
        self.epoch += 1
        G, V = self._dev_in(G_layers, "G_layers", self.L), self._dev_in(V_layers, "V_layers", self.L)
        scal, (g, h) = self._dev_out(2, self.L)
        check(lib.qhvp_hvp_ti_dev(self.handle, G.data_ptr(), V.data_ptr(), int(riemannian), scal.data_ptr(),
                                  scal.data_ptr() + 8, g.data_ptr(), h.data_ptr()))
        self._dev_keep = (G, V)
        return scal[0], scal[1], g, h

    def overlaps(self):
        T = np.empty(self.n_samples, dtype=np.complex128)
        O = np.empty(self.n_samples, dtype=np.complex128)
        check(lib.qhvp_overlaps(self.handle, dptr(_f64(T)), dptr(_f64(O))))
        return T, O

    def info(self):
        K, npass, seg = C.c_int(), C.c_int(), C.c_int()
        ws = C.c_size_t()
        check(lib.qhvp_problem_info(self.handle, C.byref(K), C.byref(npass), C.byref(ws), C.byref(seg)))
        return {"K": K.value, "n_passes": npass.value, "ws_bytes": ws.value, "segments": seg.value}

    KERNEL_KINDS = ("forward", "recompute", "backward", "reduce")

    def set_profiling(self, on: bool = True):
        check(lib.qhvp_set_profiling(self.handle, int(on)))

    def kernel_stats(self):
        out = {}
        for k, name in enumerate(self.KERNEL_KINDS):
            ms, nb, fl = C.c_double(), C.c_double(), C.c_double()
            cnt = C.c_longlong()
            check(lib.qhvp_kernel_stats(self.handle, k, C.byref(ms), C.byref(cnt), C.byref(nb), C.byref(fl)))
            out[name] = {"ms": ms.value, "launches": cnt.value, "bytes": nb.value, "flops": fl.value}
        return out

    @property
    def last_device_ms(self) -> float:
        return lib.qhvp_last_device_ms(self.handle)

    @property
    def backward_from_outputs(self) -> bool:
        """Whether the last gradient / HVP used the backward sweep from pass outputs (inverse gates)."""
        return bool(lib.qhvp_backward_from_outputs(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib.qhvp_problem_destroy(self.handle)
            self.handle = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- FP64 geometry utilities (App. F), computed in the library
def project(G, X):
    G, X = _c128(G), _c128(X)
    out = np.empty_like(G)
    check(lib.qhvp_project(G.shape[0], dptr(_f64(G)), dptr(_f64(X)), dptr(_f64(out))))
    return out


def riemannian_hvp(G, grad, hvp, V):
    G, grad, hvp, V = _c128(G), _c128(grad), _c128(hvp), _c128(V)
    out = np.empty_like(G)
    check(lib.qhvp_riemannian_hvp(G.shape[0], dptr(_f64(G)), dptr(_f64(grad)), dptr(_f64(hvp)),
                                  dptr(_f64(V)), dptr(_f64(out))))
    return out


def retract(G, xi):
    G, xi = _c128(G), _c128(xi)
    out = np.empty_like(G)
    check(lib.qhvp_retract(G.shape[0], dptr(_f64(G)), dptr(_f64(xi)), dptr(_f64(out))))
    return out


def unitarity_error(G) -> float:
    G = _c128(G)
    return float(lib.qhvp_unitarity_error(G.shape[0], dptr(_f64(G))))
