"""Serving loop: admission, chunking, overlap, fairness, failures (CPU, with a fake executor);
results alone vs in the mix and latency report (GPU)."""
import threading
import time

import numpy as np
import pytest

from oracle import circuit, sv
from paper_2604_20384_amd import serve
from paper_2604_20384_amd.inputs import make_problem


class FakeExecutor:
    """Computes results with the oracle (small n) and sleeps `delay` seconds per chunk; records
    how much memory the running requests hold."""

    def __init__(self, delay=0.02, fail_rid=None):
        from paper_2604_20384_amd.api import workspace_bytes
        self.bytes_fn = workspace_bytes
        self.delay = delay
        self.fail_rid = fail_rid
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.order = []

    def new_stream(self):
        return None

    def run_chunk(self, req, lo, hi, ckpt, stream):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            if lo == 0:
                self.order.append(req.rid)
        try:
            if req.rid == self.fail_rid:
                raise RuntimeError("injected failure")
            time.sleep(self.delay)
            psi, phi = circuit.labels(req.uref, req.samples[lo:hi], req.n, req.L_ref)
            out = sv.evaluate(psi, phi, req.G, req.V if req.kind == "hvp" else None, req.n, req.L)
            return out["fidelity"], out["grad"], out.get("hvp")
        finally:
            with self.lock:
                self.running -= 1


def _req(n, L, ns, kind, seed):
    p = make_problem(n, L, ns, seed=seed)
    return serve.Request(kind, n, L, p.uref, p.samples, p.G, p.V if kind == "hvp" else None, L_ref=p.L_ref,
                         precision="c128")


def test_results_and_fifo_and_overlap():
    ex = FakeExecutor(delay=0.05)
    srv = serve.Server(ex, slots=4, memory_budget=1 << 40)
    reqs = [_req(4 + i % 3, 2 + i % 2, 3, "hvp" if i % 2 else "grad", i) for i in range(12)]
    t0 = time.perf_counter()
    futs = [srv.submit(r) for r in reqs]
    res = [f.result() for f in futs]
    dt = time.perf_counter() - t0
    srv.shutdown()
    assert ex.order == list(range(12))              # started in arrival order
    assert ex.max_running > 1                       # requests overlapped
    assert dt < 12 * 0.05                           # faster than one at a time
    for r, q in zip(res, reqs):
        psi, phi = circuit.labels(q.uref, q.samples, q.n, q.L_ref)
        out = sv.evaluate(psi, phi, q.G, q.V, q.n, q.L)
        assert abs(r.cost - out["cost"]) < 1e-14
        assert np.allclose(r.grad, out["grad"], atol=1e-15)
        if q.kind == "hvp":
            assert np.allclose(r.hvp, out["hvp"], atol=1e-15)


def test_memory_admission_never_exceeds_budget():
    from paper_2604_20384_amd.api import workspace_bytes
    reqs = [_req(6, 3, 4, "hvp", 100 + i) for i in range(8)]
    one = workspace_bytes(6, 3, 6, 4, "c128", 0, True)
    ex = FakeExecutor(delay=0.03)
    srv = serve.Server(ex, slots=8, memory_budget=2 * one + one // 2, request_cap=one)
    [f.result() for f in [srv.submit(r) for r in reqs]]
    srv.shutdown()
    assert ex.max_running == 2                      # memory, not slots, limits the overlap


def test_sample_chunking_matches_unchunked():
    from paper_2604_20384_amd.api import workspace_bytes
    q = _req(5, 3, 9, "hvp", 7)
    full = workspace_bytes(5, 3, 6, 9, "c128", 8, True)
    cap = workspace_bytes(5, 3, 6, 3, "c128", 0, True)
    plan = serve.plan_request(q, workspace_bytes, cap)
    assert len(plan.chunks) > 1 and full > cap
    assert plan.chunks[0][0] == 0 and plan.chunks[-1][1] == 9
    srv = serve.Server(FakeExecutor(delay=0.0), slots=2, memory_budget=4 * cap, request_cap=cap)
    r = srv.submit(q).result()
    srv.shutdown()
    psi, phi = circuit.labels(q.uref, q.samples, q.n, q.L_ref)
    out = sv.evaluate(psi, phi, q.G, q.V, q.n, q.L)
    assert abs(r.fidelity - out["fidelity"]) < 1e-15
    assert np.allclose(r.grad, out["grad"], atol=1e-15) and np.allclose(r.hvp, out["hvp"], atol=1e-15)


def test_planner_takes_the_rebuilding_sweep_when_boundaries_do_not_fit():
    """Keeping every boundary when it fits the cap; else the rebuilding backward sweep if every gate
    is conditioned well enough; else the recomputing checkpoint schedules."""
    from paper_2604_20384_amd.api import workspace_bytes
    q = _req(10, 8, 16, "hvp", 11)
    keep = workspace_bytes(10, 8, 16, 16, "c128", 0, True)
    rebuild = workspace_bytes(10, 8, 16, 16, "c128", "rebuild", True)
    assert rebuild < keep
    assert serve.plan_request(q, workspace_bytes, keep).ckpt_every == 0
    p = serve.plan_request(q, workspace_bytes, rebuild)
    assert p.ckpt_every == "rebuild" and p.chunks == [(0, 16)] and p.bytes == rebuild
    G0 = q.G.copy()
    # near a unitary the bound is second order: a 1e-5 perturbation still qualifies, 1e-3 does not
    assert serve.rebuild_allowed(G0 + 1e-5)
    rng = np.random.default_rng(0)
    q.G = G0 + 1e-3 * (rng.standard_normal(G0.shape) + 1j * rng.standard_normal(G0.shape))
    assert not serve.rebuild_allowed(q.G)
    p = serve.plan_request(q, workspace_bytes, rebuild)
    assert p.ckpt_every != "rebuild"


def test_failure_is_isolated():
    ex = FakeExecutor(delay=0.01, fail_rid=2)
    srv = serve.Server(ex, slots=2, memory_budget=1 << 40)
    futs = [srv.submit(_req(4, 2, 2, "grad", i)) for i in range(5)]
    with pytest.raises(RuntimeError, match="injected"):
        futs[2].result()
    assert all(f.result().cost > 0 for i, f in enumerate(futs) if i != 2)
    srv.shutdown()


def test_oversized_request_is_rejected():
    q = _req(6, 2, 2, "grad", 1)
    srv = serve.Server(FakeExecutor(), slots=1, memory_budget=1 << 20, request_cap=1 << 10)
    with pytest.raises(MemoryError):
        srv.submit(q)
    srv.shutdown()


def test_cancel_a_queued_request():
    """A request cancelled while queued is dropped when it reaches the head, without taking memory
    or a slot; the requests around it are served."""
    ex = FakeExecutor(delay=0.05)
    srv = serve.Server(ex, slots=1, memory_budget=1 << 40)
    futs = [srv.submit(_req(4, 2, 2, "grad", i)) for i in range(4)]
    time.sleep(0.01)                                  # the first one is running by now
    assert futs[2].cancel()
    assert not futs[0].cancel()                       # a running request cannot be cancelled
    done = [futs[i].result() for i in (0, 1, 3)]
    srv.shutdown()
    assert futs[2].cancelled() and srv.cancelled == 1
    assert [r.rid for r in done] == [0, 1, 3] and 2 not in ex.order
    assert srv._free == 1 << 40                      # nothing held: the cancelled one never took memory


def test_busy_fraction():
    R = serve.Result
    res = [R(0, 0, 0, None, None, 0.0, 1.0, 3.0, None), R(1, 0, 0, None, None, 0.0, 2.0, 4.0, None),
           R(2, 0, 0, None, None, 0.0, 6.0, 7.0, None)]
    assert abs(serve.busy_fraction(res, 0.0, 10.0) - 0.4) < 1e-12


def test_latency_report_and_poisson():
    rng = np.random.default_rng(0)
    arr = serve.poisson_arrivals(rng, rate=50.0, count=2000)
    assert abs(np.mean(np.diff(arr)) - 1 / 50.0) < 0.002
    ex = FakeExecutor(delay=0.005)
    srv = serve.Server(ex, slots=2, memory_budget=1 << 40)
    reqs = [_req(4, 2, 2, "grad", i) for i in range(10)]
    res, t0, t1 = serve.replay(srv, reqs, serve.poisson_arrivals(rng, 100.0, 10))
    srv.shutdown()
    rep = serve.latency_report(res, t0, t1)
    assert rep["requests"] == 10 and rep["p99_s"] >= rep["p50_s"] > 0


@pytest.mark.gpu
def test_gpu_results_alone_equal_results_in_the_mix(gpu):
    """Mixed n / L / N_s grad and HVP requests overlap on four streams; every result is bitwise
    the result of the same request served alone."""
    rng = np.random.default_rng(3)
    reqs = [serve.random_request(rng, n_range=(10, 16), L_range=(2, 8), ns_range=(4, 48)) for _ in range(16)]
    ex = serve.GpuExecutor()
    srv = serve.Server(ex, slots=4, memory_budget=64 << 30)
    res, t0, t1 = serve.replay(srv, reqs, serve.poisson_arrivals(rng, 200.0, len(reqs)))
    srv.shutdown()
    alone = serve.Server(serve.GpuExecutor(), slots=1, memory_budget=64 << 30)
    for q, r in zip(reqs, res):
        a = alone.submit(q).result()
        assert a.cost == r.cost and np.array_equal(a.grad, r.grad)
        if q.kind == "hvp":
            assert np.array_equal(a.hvp, r.hvp)
    alone.shutdown()
    rep = serve.latency_report(res, t0, t1)
    print("served:", rep)
    assert rep["requests"] == 16


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("c128", 1e-10), ("c64", 1e-5)])
def test_gpu_chunked_request_against_oracle(gpu, precision, tol):
    """A request whose workspace exceeds the per-request cap is split into sample chunks on the GPU;
    the sample-weighted sum of the chunks' results equals the oracle over all samples."""
    from parity import assert_close, assert_fidelity
    from paper_2604_20384_amd.api import workspace_bytes
    p = make_problem(10, 4, 9, seed=91)
    q = serve.Request("hvp", 10, 4, p.uref, p.samples, p.G, p.V, L_ref=p.L_ref, precision=precision)
    cap = workspace_bytes(10, 4, 8, 3, precision, 0, True)
    plan = serve.plan_request(q, workspace_bytes, cap)
    assert len(plan.chunks) >= 2, plan
    srv = serve.Server(serve.GpuExecutor(), slots=2, memory_budget=4 * cap, request_cap=cap)
    r = srv.submit(q).result()
    srv.shutdown()
    psi, phi = circuit.labels(p.uref, p.samples, p.n, p.L_ref)
    ref = sv.evaluate(psi, phi, p.G, p.V, p.n, p.L)
    assert_fidelity(r.fidelity, ref["fidelity"], tol, "chunked")
    assert_close(r.grad, ref["grad"], tol, "chunked grad")
    assert_close(r.hvp, ref["hvp"], tol, "chunked hvp")


def test_arena_first_fit_and_coalescing():
    a = serve.Arena(4096, base_ptr=1 << 20)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048) and a.alloc(2000) is None
    a.free(y)
    assert a.alloc(1100) is None and a.alloc(900) == 1024
    a.free(1024)
    a.free(x)
    a.free(z)
    assert a.free_list == [(0, 4096)] and a.largest_free() == 4096
