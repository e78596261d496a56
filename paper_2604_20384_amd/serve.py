"""Continuous-batching server for gradient / HVP requests of mixed size.

Requests (n, L, N_s, U_ref, samples, G, V) arrive at any time.  A fixed number of slots, each
with its own HIP stream, take requests from a FIFO queue as soon as a slot is free and the
request's device memory fits into what is left of the memory budget; the work of all running
requests then overlaps on the GPU (one host thread per slot drives the library, which releases
the GIL).  Each request is planned from its own shape only: the layer-checkpoint interval and, if
even the leanest plan exceeds the per-request cap, a split of its samples into chunks whose
sample-weighted results are added (the cost, gradient and HVP are averages over independent
samples, Sec. IV).  A request's result therefore does not depend on what else is running; the
kernels reduce in a fixed order, so it is bitwise the same alone and in the mix.

Latency = completion time - arrival time (including the request's label sweep
phi_s = U_ref psi_s, which every new request needs).  A queued request can be cancelled through its
future (Future.cancel) until a slot takes it; the others are not held up.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from concurrent.futures import Future

import numpy as np

# checkpoint policies from fastest (most memory) to leanest; "rebuild" (only the final forward
# states kept, the backward sweep rebuilds the pass boundaries) needs well-conditioned gates
CKPT_CHOICES = (0, "rebuild", -2, 1, 2, 4, 8)
# The device accepts "rebuild" for gates with |G|_F |G^-1|_F <= 4 (1 + 1e-6); the planner asks for a
# little less, so that no rounding difference between the two checks can make a planned request fail.
REBUILD_COND = 4.0 * (1.0 + 0.5e-6)


def rebuild_allowed(G: np.ndarray) -> bool:
    """Whether every gate is conditioned well enough for the rebuilding sweep (the device's test)."""
    G = np.asarray(G, dtype=np.complex128)
    try:
        Gi = np.linalg.inv(G)
    except np.linalg.LinAlgError:
        return False
    prod = np.linalg.norm(G, axis=(1, 2)) * np.linalg.norm(Gi, axis=(1, 2))
    return bool(np.all(prod <= REBUILD_COND))


@dataclasses.dataclass
class Request:
    kind: str                      # "grad" or "hvp"
    n: int
    L: int
    uref: np.ndarray               # (K_ref, 4, 4)
    samples: np.ndarray            # (N_s, n, 2)
    G: np.ndarray                  # (K, 4, 4)
    V: np.ndarray | None = None    # (K, 4, 4) for "hvp"
    L_ref: int | None = None
    precision: str = "c64"
    rid: int = -1
    arrival: float = 0.0

    @property
    def n_samples(self) -> int:
        return self.samples.shape[0]


@dataclasses.dataclass
class Plan:
    ckpt_every: int | str          # a checkpoint interval, or "rebuild"
    chunks: list                   # list of (start, stop) sample ranges
    bytes: int                     # device memory held while the request runs (largest chunk)


@dataclasses.dataclass
class Result:
    rid: int
    cost: float
    fidelity: float
    grad: np.ndarray
    hvp: np.ndarray | None
    arrival: float
    start: float
    end: float
    plan: Plan

    @property
    def latency(self) -> float:
        return self.end - self.arrival


def plan_request(req: Request, bytes_fn, cap: int) -> Plan:
    """Fastest checkpoint policy whose workspace fits `cap`; split the samples in 2, 4, ...
    chunks if none does.  Depends on the request only (its shape, and its gates for "rebuild")."""
    Lr = req.L_ref if req.L_ref is not None else 2 * req.L
    ns = req.n_samples
    tangent = req.kind == "hvp"
    choices = [ck for ck in CKPT_CHOICES if ck != "rebuild" or rebuild_allowed(req.G)]
    chunks = 1
    while True:
        size = math.ceil(ns / chunks)
        for ck in choices:
            b = bytes_fn(req.n, req.L, Lr, size, req.precision, ck, tangent)
            if 0 < b <= cap:
                rng = [(i, min(ns, i + size)) for i in range(0, ns, size)]
                return Plan(ck, rng, b)
        if size == 1:
            raise MemoryError(f"request {req.rid}: even one sample needs more than {cap} bytes")
        chunks *= 2


class Arena:
    """First-fit allocator over one device buffer that is allocated once (from torch, so its HBM
    shows in torch's statistics).  Blocks are 256-byte aligned offsets; not thread-safe (the
    server calls it under its lock)."""

    ALIGN = 256

    def __init__(self, nbytes: int, device: int = 0, base_ptr: int | None = None):
        self.size = nbytes
        self.buf = None
        if base_ptr is None:
            import torch
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
            base_ptr = self.buf.data_ptr()
        self.base = base_ptr
        self.free_list = [(0, nbytes)]          # sorted, coalesced (offset, size)
        self.used = {}

    def alloc(self, nbytes: int):
        need = (nbytes + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for i, (off, sz) in enumerate(self.free_list):
            if sz >= need:
                if sz == need:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + need, sz - need)
                self.used[off] = need
                return off
        return None

    def free(self, off: int):
        need = self.used.pop(off)
        self.free_list.append((off, need))
        self.free_list.sort()
        merged = []
        for o, z in self.free_list:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + z)
            else:
                merged.append((o, z))
        self.free_list = merged

    def largest_free(self) -> int:
        return max((z for _, z in self.free_list), default=0)


class GpuExecutor:
    """Runs requests through the HIP library (paper_2604_20384_amd.api), each in a block of the
    server's device arena."""

    def __init__(self, device: int = 0):
        self.device = device

    def make_arena(self, nbytes: int) -> Arena:
        return Arena(nbytes, self.device)

    def bytes_fn(self, n, L, L_ref, ns, precision, ckpt, tangent):
        from .api import workspace_bytes
        return workspace_bytes(n, L, L_ref, ns, precision, ckpt, tangent)

    def new_stream(self):
        import torch
        return torch.cuda.Stream(device=self.device)

    def run_chunk(self, req: Request, lo: int, hi: int, ckpt: int, stream, workspace=None):
        """Returns (fidelity, grad, hvp) averaged over samples lo..hi-1; `workspace` is a
        (device pointer, bytes) block."""
        import torch

        from .api import Problem
        Lr = req.L_ref if req.L_ref is not None else 2 * req.L
        with torch.cuda.stream(stream):
            p = Problem(req.n, req.L, req.uref, req.samples[lo:hi], L_ref=Lr, precision=req.precision,
                        ckpt_every=ckpt, with_tangent=req.kind == "hvp", device=self.device, stream=stream,
                        workspace=workspace if workspace is not None else "torch")
            try:
                if req.kind == "hvp":
                    c, g, h = p.hvp(req.G, req.V)
                else:
                    c, g = p.grad(req.G)
                    h = None
                F = p.last_fidelity       # as computed (1 - c cancels when F is small)
            finally:
                p.close()
        return F, g, h


class Server:
    def __init__(self, executor, slots: int = 4, memory_budget: int = 200 << 30,
                 request_cap: int | None = None):
        self.ex = executor
        self.slots = slots
        self.budget = memory_budget
        self.cap = request_cap if request_cap is not None else memory_budget // 2
        self._q = collections.deque()
        self._cv = threading.Condition()
        self._free = memory_budget
        self.arena = executor.make_arena(memory_budget) if hasattr(executor, "make_arena") else None
        self._stop = False
        self._next_id = 0
        self.results: list[Result] = []
        self.busy_s = 0.0
        self.cancelled = 0
        self._threads = []
        for i in range(slots):
            t = threading.Thread(target=self._worker, args=(i,), daemon=True)
            t.start()
            self._threads.append(t)

    def submit(self, req: Request, arrival: float | None = None) -> Future:
        fut: Future = Future()
        with self._cv:
            req.rid = self._next_id if req.rid < 0 else req.rid
            self._next_id += 1
            req.arrival = time.perf_counter() if arrival is None else arrival
            plan = plan_request(req, self.ex.bytes_fn, self.cap)
            self._q.append((req, plan, fut))
            self._cv.notify_all()
        return fut

    def _take(self):
        """FIFO head, once its memory fits (head-of-line blocking keeps the order fair).  Cancelled
        requests are dropped when they reach the head, before any memory is taken for them."""
        with self._cv:
            while True:
                if self._stop and not self._q:
                    return None
                while self._q and self._q[0][2].cancelled():
                    self._q.popleft()
                    self.cancelled += 1
                if self._q:
                    nbytes = self._q[0][1].bytes
                    if self.arena is not None:
                        off = self.arena.alloc(nbytes)
                        if off is not None:
                            return self._q.popleft() + (off,)
                    elif nbytes <= self._free:
                        self._free -= nbytes
                        return self._q.popleft() + (None,)
                self._cv.wait(0.05)

    def _release(self, nbytes, off):
        with self._cv:
            if off is not None:
                self.arena.free(off)
            else:
                self._free += nbytes
            self._cv.notify_all()

    def _worker(self, slot: int):
        stream = self.ex.new_stream()
        while True:
            item = self._take()
            if item is None:
                return
            req, plan, fut, off = item
            if not fut.set_running_or_notify_cancel():     # cancelled after it was taken
                with self._cv:
                    self.cancelled += 1
                self._release(plan.bytes, off)
                continue
            ws = None if off is None else (self.arena.base + off, plan.bytes)
            t0 = time.perf_counter()
            try:
                F = 0.0
                g = np.zeros_like(req.G, dtype=np.complex128)
                h = np.zeros_like(req.G, dtype=np.complex128) if req.kind == "hvp" else None
                ns = req.n_samples
                for lo, hi in plan.chunks:
                    if ws is None:
                        f_c, g_c, h_c = self.ex.run_chunk(req, lo, hi, plan.ckpt_every, stream)
                    else:
                        f_c, g_c, h_c = self.ex.run_chunk(req, lo, hi, plan.ckpt_every, stream, workspace=ws)
                    w = (hi - lo) / ns
                    F += w * f_c
                    g += w * g_c
                    if h is not None:
                        h += w * h_c
                t1 = time.perf_counter()
                res = Result(req.rid, 1.0 - F, F, g, h, req.arrival, t0, t1, plan)
                with self._cv:
                    self.results.append(res)
                    self.busy_s += t1 - t0
                fut.set_result(res)
            except BaseException as e:  # the request fails, the server keeps going
                fut.set_exception(e)
            finally:
                self._release(plan.bytes, off)

    def shutdown(self, wait: bool = True):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        if wait:
            for t in self._threads:
                t.join()
            self.arena = None          # release the device buffer


def busy_fraction(results, t_start: float, t_end: float) -> float:
    """Share of [t_start, t_end] during which at least one request was running (the union of the
    requests' start..end intervals; each request keeps the device working from start to end)."""
    spans = sorted((r.start, r.end) for r in results)
    busy, cur_s, cur_e = 0.0, None, None
    for s0, e0 in spans:
        s0, e0 = max(s0, t_start), min(e0, t_end)
        if cur_e is None or s0 > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    if cur_e is not None:
        busy += cur_e - cur_s
    return busy / max(1e-9, t_end - t_start)


def latency_report(results, t_start: float, t_end: float) -> dict:
    lat = np.array([r.latency for r in results])
    return {
        "requests": len(results),
        "throughput_rps": len(results) / max(1e-9, t_end - t_start),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_s": float(lat.mean()) if len(lat) else None,
        "busy_frac": busy_fraction(results, t_start, t_end) if len(lat) else None,
    }


def poisson_arrivals(rng: np.random.Generator, rate: float, count: int) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def replay(server: Server, requests, arrivals) -> tuple[list, float, float]:
    """Submit `requests` at the given offsets (seconds from now); wait for all; return results."""
    t0 = time.perf_counter()
    futs = []
    for req, at in zip(requests, arrivals):
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        futs.append(server.submit(req, arrival=t0 + at))
    res = [f.result() for f in futs]
    return res, t0, time.perf_counter()


def random_request(rng: np.random.Generator, n_range=(10, 22), L_range=(4, 32), ns_range=(16, 256),
                   kinds=("grad", "hvp"), precision="c64") -> Request:
    """A synthetic request: Haar gates, Haar U_ref of depth 2L, Haar product samples, tangent V."""
    from .inputs import make_problem
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    L = int(rng.integers(L_range[0], L_range[1] + 1))
    ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
    kind = str(rng.choice(kinds))
    p = make_problem(n, L, ns, seed=int(rng.integers(0, 2 ** 31)))
    return Request(kind, n, L, p.uref, p.samples, p.G, p.V if kind == "hvp" else None, L_ref=p.L_ref,
                   precision=precision)
