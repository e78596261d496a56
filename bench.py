"""Benchmark: Hessian-vector products per second of the brickwall Hilbert-Schmidt cost at
n=20 qubits, L=20 layers (K=190 gates), N_s=256 Haar product samples, U_ref a Haar brickwall
of depth 40, complex64 states with FP64 accumulation, on one MI355X.

One step = one from-scratch HVP call (cost + gradient + HVP for one (G, V) over all samples),
each at its own Haar G, so that no forward state kept from an earlier call belongs to it; the
labels phi_s = U_ref psi_s are computed once per problem (the problem statement takes them as
input) and reported separately as setup time.  Further legs, reported beside the headline figure:

* fixed_G: HVPs along several directions at one G (the forward states at G are kept between calls);
* ckpt4: the headline workload with layer checkpointing every 4 layers (rate and peak HBM);
* rebuild: the headline workload keeping only the final forward states, the backward sweep
  rebuilding every pass boundary by undoing the pass's gates (rate and peak HBM);
* c128: the same workload in complex128, with its own roofline against the FP64 peak;
* ti: the translationally invariant ansatz (one gate per layer, per-layer outputs, App. E);
* accuracy: fidelity, gradient and HVP errors against the oracle on samples 0-3 (both precisions)
  and complex64 against complex128 on all 256 samples, globally and gate by gate;
* serving: a Poisson stream of mixed gradient / HVP requests (n 10-22, L 4-32, N_s 16-256,
  complex64) at rates swept over 0.25-1.2x the measured serial capacity, served one at a time and
  with continuous batching, with throughput, p50 / p99 latency and GPU-busy fraction;
* cpu_baseline: the oracle on the host, one single-threaded process per sample for samples 0-3 run
  together (the same runs give the accuracy reference);
* c2: the n=16, L=12, N_s=64 problem on the GPU in both precisions, and whole on P single-threaded
  oracle processes, timed directly, with the GPU results' errors against that oracle run.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# Compute peaks of the unit that executes the arithmetic of each precision: complex64 runs the gate
# products and the environment sums on the FP32 matrix cores (dense MFMA FP32: 157.3 TFLOP/s);
# complex128 runs the gate products on the FP64 vector ALU and the sums on FP64 MFMA, both 78.6.
COMPUTE_PEAK = {"c64": ("mfma", 157.3), "c128": ("alu", 78.6)}
TRAFFIC_PROFILE = "profiles/traffic_k_bwd_out_c64.json"
ORACLE_SAMPLES = 4
MAX_HOST_WORKERS = 16          # host processes of the n=16 oracle run (the host share of one GPU)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--L", type=int, default=20)
    ap.add_argument("--ns", type=int, default=256)
    ap.add_argument("--precision", default="c64", choices=["c64", "c128"])
    ap.add_argument("--ckpt", type=lambda v: v if v == "rebuild" else int(v), default=None,
                    help="layer checkpoint interval (0: every pass boundary; 'rebuild': only the final "
                         "states, the backward sweep rebuilds the boundaries; default: the fastest that fits)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 2 GiB device copy 5 times (calibrates HBM traffic counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle runs (and the accuracy leg)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the accuracy, ckpt4, ti and c128 legs")
    ap.add_argument("--serve-requests", type=int, default=40, help="requests per arrival rate")
    ap.add_argument("--serve-rates", default="0.25,0.5,0.75,0.9,1.0,1.2",
                    help="arrival rates as multiples of the measured serial capacity")
    ap.add_argument("--fixed-g-dirs", type=int, default=8,
                    help="directions of the fixed-G leg (0: skip it)")
    ap.add_argument("--seed", type=int, default=1)
    return ap.parse_args()


# ---------------------------------------------------------------------------------------------
# the oracle on the host (test infrastructure: timed as the CPU baseline, and the accuracy reference)

def _oracle_sample(job):
    """One sample of the workload through the numpy complex128 oracle, single-threaded."""
    n, L, ns, seed, s = job
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import circuit, sv
    from paper_2604_20384_amd.inputs import make_problem
    with threadpool_limits(1):
        p = make_problem(n, L, ns, seed=seed)
        psi, phi = circuit.labels(p.uref, p.samples[s:s + 1], n, p.L_ref)
        t0 = time.perf_counter()
        out = sv.evaluate(psi, phi, p.G, p.V, n, L, batch=1)
        dt = time.perf_counter() - t0
    return dt, float(out["fidelity"]), np.asarray(out["grad"]), np.asarray(out["hvp"])


def oracle_pool():
    """ORACLE_SAMPLES worker processes, started before this process touches the GPU (so that no
    process that holds the GPU starts another program); they wait for work."""
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(ORACLE_SAMPLES)


def start_oracle(pool, n, L, ns, seed):
    """Samples 0..ORACLE_SAMPLES-1, one per worker."""
    return pool, pool.map_async(_oracle_sample, [(n, L, ns, seed, s) for s in range(ORACLE_SAMPLES)])


# The configuration the oracle runs whole: n=16, L=12 (K=90), L_ref=24, N_s=64.
C2 = (16, 12, 64)


def _c2_worker(rank, P, seed, go, barrier, q):
    """Samples rank, rank+P, ... of the n=16 problem through the oracle, single-threaded: labels
    first, then (once all P workers are ready) the timed evaluation."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import circuit, sv
    from paper_2604_20384_amd.inputs import make_problem
    n, L, ns = C2
    if not go.wait(3600):
        return
    with threadpool_limits(1):
        p = make_problem(n, L, ns, seed=seed)
        mine = list(range(rank, ns, P))
        psi, phi = circuit.labels(p.uref, p.samples[mine], n, p.L_ref)
        barrier.wait(600)
        t0 = time.time()
        out = sv.evaluate(psi, phi, p.G, p.V, n, L, batch=1)
        t1 = time.time()
    # sample-weighted, so that the parent adds the parts of all workers
    w = len(mine)
    q.put((rank, t0, t1, w * float(out["fidelity"]), w * np.asarray(out["grad"]), w * np.asarray(out["hvp"])))


def c2_oracle_start(seed):
    """P = the host cores this process may use (at most MAX_HOST_WORKERS); P worker processes,
    started before this process touches the GPU, wait until c2_oracle_run releases them."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    P = min(MAX_HOST_WORKERS, len(os.sched_getaffinity(0)))
    go, barrier, q = ctx.Event(), ctx.Barrier(P), ctx.Queue()
    procs = [ctx.Process(target=_c2_worker, args=(r, P, seed, go, barrier, q), daemon=True) for r in range(P)]
    for pr in procs:
        pr.start()
    # the handle keeps every shared object alive: a child unpickles them after start() returns
    return P, go, barrier, q, procs


def c2_oracle_run(handle):
    """The full n=16 problem on P single-threaded processes, timed directly: from the first worker's
    start of the evaluation to the last one's end (labels excluded, as on the GPU)."""
    import numpy as np
    P, go, _barrier, q, procs = handle
    go.set()
    parts = [q.get(timeout=900) for _ in range(P)]
    for pr in procs:
        pr.join(60)
    wall = max(r[2] for r in parts) - min(r[1] for r in parts)
    ns = C2[2]
    ref = (sum(r[3] for r in parts) / ns, sum(r[4] for r in parts) / ns, sum(r[5] for r in parts) / ns)
    return P, wall, (float(ref[0]), np.asarray(ref[1]), np.asarray(ref[2]))


def c2_gpu_leg(seed, timed=10, warmup=3):
    """The n=16 problem on the GPU in both precisions: from-scratch HVPs (a fresh Haar G per call),
    median of `timed` individually timed calls after `warmup`; plus one call at the problem's own
    (G, V) for the accuracy against the oracle."""
    import numpy as np
    import torch

    from paper_2604_20384_amd.api import Problem, num_gates
    from paper_2604_20384_amd.inputs import haar_unitary, make_problem, random_tangent
    n, L, ns = C2
    prob = make_problem(n, L, ns, seed=seed)
    rng = np.random.default_rng(seed + 5000)
    K = num_gates(n, L)
    Gs = [haar_unitary(rng, 4, K) for _ in range(warmup + timed)]
    Vs = [random_tangent(rng, G) for G in Gs]
    out, results = {}, {}
    for precision in ("c64", "c128"):
        gp = Problem(n, L, prob.uref, prob.samples, L_ref=prob.L_ref, precision=precision, ckpt_every=0, device=0)
        times = []
        for i in range(warmup + timed):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gp.hvp(Gs[i], Vs[i])
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        med = float(np.median(times[warmup:]))
        _, g, h = gp.hvp(prob.G, prob.V)
        results[precision] = (gp.last_fidelity, g, h)
        gp.close()
        out[precision] = {"value": round(1.0 / med, 2), "unit": "HVP/s", "median_ms": round(1e3 * med, 3),
                          "timed_calls": timed, "ckpt_every_layers": 0}
    return out, results


def cpu_info():
    import subprocess

    from threadpoolctl import threadpool_info
    model = ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    blas = [f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()]
    return model, blas


# ---------------------------------------------------------------------------------------------

def kernel_source_sha256():
    """sha256 of the sweep kernels' source and the shared header that fixes their layouts."""
    import hashlib
    h = hashlib.sha256()
    for name in ("qhvp_kernels.hip", "qhvp_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2604_20384_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if the kernel source has changed
    since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    try:
        rec = json.load(open(path))
        sha = kernel_source_sha256()
    except OSError:
        return None, None
    if rec.get("kernel") != kernel_name or not sha.startswith(rec["kernel_source_sha256_prefix"]):
        return None, rec
    b = (rec["fetch_kib_per_launch"] * rec["fetch_factor"] + rec["write_kib_per_launch"] * rec["write_factor"]) * 1024
    return b, rec


def copy_probe():
    import torch
    nbytes = 2 << 30
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}))


def pick_ckpt(n, L, L_ref, ns, precision, choices=(0, -2, 1, 2, 4, 8)):
    """Fastest checkpoint policy whose workspace fits the free HBM (8 GiB kept back)."""
    import torch

    from paper_2604_20384_amd.api import workspace_bytes
    free, _ = torch.cuda.mem_get_info()
    for ck in choices:
        if workspace_bytes(n, L, L_ref, ns, precision, ck, True) <= free - (8 << 30):
            return ck
    return choices[-1]


def timed_hvps(gp, Gs, Vs, warmup, steps):
    """`warmup` untimed then `steps` timed HVPs; returns (seconds, kernel stats of the timed ones)."""
    import torch
    for i in range(warmup):
        gp.hvp(Gs[i], Vs[i])
    gp.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        gp.hvp(Gs[i], Vs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = gp.kernel_stats()
    gp.set_profiling(False)
    return dt, stats


def roofline(stats, precision, steps, gp, with_traffic):
    """The dominant kernel (most device time) against its roofline."""
    dom = max(("forward", "recompute", "backward"), key=lambda k: stats[k]["ms"])
    st = stats[dom]
    avg_ms = st["ms"] / max(1, st["launches"])
    bytes_per_launch = st["bytes"] / max(1, st["launches"])
    flops_per_launch = st["flops"] / max(1, st["launches"])
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    tfs = flops_per_launch / (avg_ms * 1e-3) / 1e12
    unit_name, comp_peak = COMPUTE_PEAK[precision]
    frac_hbm, frac_comp = gbs / HBM_PEAK_GBS, tfs / comp_peak
    if frac_hbm >= frac_comp:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(frac_hbm, 4)}
    else:
        roof = {"bound": unit_name, "achieved": round(tfs, 2), "peak": comp_peak, "unit": "TFLOP/s",
                "frac": round(frac_comp, 4)}
    rt = "float" if precision == "c64" else "double"
    bwd_name = "k_bwd_out" if gp.backward_from_outputs else "k_bwd"
    kname = f"{bwd_name}<{rt},true>" if dom == "backward" else f"k_fwd<{rt},true>"
    traffic, rec = measured_traffic(kname) if with_traffic else (None, None)
    roof.update({"traffic": traffic, "kernel": kname, "avg_launch_ms": round(avg_ms, 4), "launches": st["launches"],
                 "alg_bytes_per_launch": bytes_per_launch, "alg_flops_per_launch": flops_per_launch,
                 "hbm_frac": round(frac_hbm, 4), "compute_frac": round(frac_comp, 4),
                 "compute_peak_TFLOPs": comp_peak})
    if with_traffic:
        roof["traffic_source"] = (
            f"{TRAFFIC_PROFILE}: rocprofv3 FETCH_SIZE x {rec['fetch_factor']} + WRITE_SIZE x {rec['write_factor']} "
            "(factors from a copy kernel of known size), per launch; null when the kernel source changed since"
            if rec else "no committed counter profile")
    return roof


def fixed_g_leg(gp, G, M, rng, from_scratch_hvps):
    """HVPs along M directions at one G (hvp_batch) after a gradient call at G, so every direction
    reads the kept forward states at G and stores only tangents."""
    import numpy as np
    import torch

    from paper_2604_20384_amd.inputs import random_tangent
    Vfix = np.stack([random_tangent(rng, G) for _ in range(M)])
    gp.grad(G)
    gp.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gp.hvp_batch(G, Vfix)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = gp.kernel_stats()
    gp.set_profiling(False)
    return {"directions": M, "value": round(M / dt, 4), "unit": "HVP/s", "ms_per_hvp": round(1e3 * dt / M, 3),
            "kernel_ms_per_hvp": {k: round(v["ms"] / M, 3) for k, v in stats.items()},
            "alg_bytes_per_hvp": sum(v["bytes"] for v in stats.values()) / M,
            "vs_from_scratch": round(M / dt / from_scratch_hvps, 4)}


def errors(got, ref):
    """Relative errors of (F, grad, hvp): global and worst gate (max |d_k| / max |ref_k|)."""
    import numpy as np

    def pg(a, b):
        a, b = np.asarray(a).reshape(-1, 16), np.asarray(b).reshape(-1, 16)
        return float(np.max(np.max(np.abs(a - b), axis=1) / np.max(np.abs(b), axis=1)))
    (F, g, h), (Fr, gr, hr) = got, ref
    return {"F": float(abs(F - Fr) / Fr),
            "grad": float(np.linalg.norm(g - gr) / np.linalg.norm(gr)), "grad_per_gate": pg(g, gr),
            "hvp": float(np.linalg.norm(h - hr) / np.linalg.norm(hr)), "hvp_per_gate": pg(h, hr)}


def one_hvp(prob, precision, ckpt, ns=None):
    """(F, grad, hvp) of one HVP at the problem's own (G, V) on a fresh GPU problem."""
    import torch

    from paper_2604_20384_amd.api import Problem
    ns = prob.n_samples if ns is None else ns
    torch.cuda.empty_cache()
    gp = Problem(prob.n, prob.L, prob.uref, prob.samples[:ns], L_ref=prob.L_ref, precision=precision,
                 ckpt_every=ckpt, device=0)
    _, g, h = gp.hvp(prob.G, prob.V)
    F = gp.last_fidelity
    gp.close()
    return F, g, h


def leg(prob, precision, ckpt, steps, rng_seed):
    """A timed leg on a fresh problem: HVP/s, peak HBM, dominant-kernel roofline."""
    import numpy as np
    import torch

    from paper_2604_20384_amd.api import Problem, num_gates
    from paper_2604_20384_amd.inputs import haar_unitary, random_tangent
    rng = np.random.default_rng(rng_seed)
    K = num_gates(prob.n, prob.L)
    Gs = [haar_unitary(rng, 4, K) for _ in range(steps + 1)]
    Vs = [random_tangent(rng, G) for G in Gs]
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    gp = Problem(prob.n, prob.L, prob.uref, prob.samples, L_ref=prob.L_ref, precision=precision,
                 ckpt_every=ckpt, device=0)
    dt, stats = timed_hvps(gp, Gs, Vs, 1, steps)
    peak = torch.cuda.max_memory_allocated() - base
    out = {"value": round(steps / dt, 4), "unit": "HVP/s", "ms_per_hvp": round(1e3 * dt / steps, 3),
           "precision": precision, "ckpt_every_layers": ckpt, "steps": steps,
           "peak_hbm_GiB": round(peak / 2 ** 30, 2),
           "kernel_ms_per_hvp": {k: round(v["ms"] / steps, 3) for k, v in stats.items()},
           "roofline": roofline(stats, precision, steps, gp, with_traffic=False)}
    gp.close()
    return out


def ti_leg(prob, steps, rng_seed, headline_hvps):
    """Translationally invariant ansatz (App. E) at the headline setting: one Haar gate and one
    tangent direction per layer, from-scratch HVP calls with per-layer outputs.  The layer gates
    are expanded and the per-layer sums taken on the device, so the rate should equal the
    headline rate."""
    import numpy as np
    import torch

    from paper_2604_20384_amd.api import Problem
    from paper_2604_20384_amd.inputs import haar_unitary, random_tangent
    rng = np.random.default_rng(rng_seed)
    Gs = [haar_unitary(rng, 4, prob.L) for _ in range(steps + 1)]
    Vs = [random_tangent(rng, G) for G in Gs]
    torch.cuda.empty_cache()
    gp = Problem(prob.n, prob.L, prob.uref, prob.samples, L_ref=prob.L_ref, precision="c64", ckpt_every=0,
                 device=0)
    gp.hvp_ti(Gs[0], Vs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(1, steps + 1):
        gp.hvp_ti(Gs[i], Vs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gp.close()
    return {"value": round(steps / dt, 4), "unit": "HVP/s", "ms_per_hvp": round(1e3 * dt / steps, 3),
            "steps": steps, "precision": "c64", "ckpt_every_layers": 0,
            "vs_headline": round(steps / dt / headline_hvps, 4),
            "note": f"{prob.L} layer gates, per-layer gradient and HVP (App. E)"}


def serving_sweep(n_req, rate_factors, seed):
    """Poisson streams of mixed gradient / HVP requests (complex64; n 10-22, L 4-32, N_s 16-256),
    at rates swept as multiples of the measured serial capacity mu: each rate's stream served one
    request at a time (FIFO, one slot) and with continuous batching (4 slots) on the same arrivals."""
    import numpy as np
    import torch

    from paper_2604_20384_amd import serve
    rng = np.random.default_rng(seed)
    reqs = [serve.random_request(rng, n_range=(10, 22), L_range=(4, 32), ns_range=(16, 256)) for _ in range(n_req)]
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(200 << 30, free - (24 << 30))) // 256 * 256
    cfg = {"requests_per_rate": n_req, "n": [10, 22], "L": [4, 32], "N_s": [16, 256], "kinds": ["grad", "hvp"],
           "precision": "c64", "memory_budget_GiB": round(budget / 2 ** 30, 1), "batched_slots": 4}
    # warm-up (first launches), then the serial capacity with every request queued at once
    w = serve.Server(serve.GpuExecutor(), slots=1, memory_budget=budget)
    w.submit(reqs[0]).result()
    w.shutdown()
    srv = serve.Server(serve.GpuExecutor(), slots=1, memory_budget=budget)
    res, t0, t1 = serve.replay(srv, reqs, np.zeros(n_req))
    srv.shutdown()
    mu = n_req / (t1 - t0)
    cfg["serial_capacity_rps"] = round(mu, 3)
    cfg["chunked_requests"] = sum(1 for r in res if len(r.plan.chunks) > 1)
    rates = []
    for f in rate_factors:
        lam = f * mu
        arrivals = serve.poisson_arrivals(rng, lam, n_req)
        row = {"rate_factor": f, "arrival_rps": round(lam, 3)}
        for name, slots in (("serial", 1), ("batched", 4)):
            srv = serve.Server(serve.GpuExecutor(), slots=slots, memory_budget=budget)
            res, t0, t1 = serve.replay(srv, reqs, arrivals)
            srv.shutdown()
            rep = serve.latency_report(res, t0, t1)
            row[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
        rates.append(row)
        print(f"serving rate {f} mu: serial p50/p99 {row['serial']['p50_s']}/{row['serial']['p99_s']} "
              f"batched {row['batched']['p50_s']}/{row['batched']['p99_s']}", file=sys.stderr, flush=True)
    cfg["rates"] = rates
    return cfg


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (--gpus must be 1): the library has no multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    pool = None if args.no_cpu_baseline else oracle_pool()
    c2_cpu = None if args.no_cpu_baseline else c2_oracle_start(args.seed)

    import numpy as np
    import torch

    from paper_2604_20384_amd.api import Problem, num_gates
    from paper_2604_20384_amd.inputs import haar_unitary, make_problem, random_tangent

    n, L, ns = args.n, args.L, args.ns
    K = num_gates(n, L)
    prob = make_problem(n, L, ns, seed=args.seed)
    # a fresh Haar G and tangent V for every call: each timed HVP is from scratch
    rng = np.random.default_rng(args.seed + 1000)
    Gs = [prob.G] + [haar_unitary(rng, 4, K) for _ in range(args.warmup + args.steps - 1)]
    Vs = [prob.V] + [random_tangent(rng, G) for G in Gs[1:]]
    if args.ckpt is None:
        args.ckpt = pick_ckpt(n, L, prob.L_ref, ns, args.precision)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    gp = Problem(n, L, prob.uref, prob.samples, L_ref=prob.L_ref, precision=args.precision,
                 ckpt_every=args.ckpt, device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    dt, stats = timed_hvps(gp, Gs, Vs, args.warmup, args.steps)
    peak_mem = torch.cuda.max_memory_allocated()
    hvps = args.steps / dt
    ms_per_step = 1e3 * dt / args.steps
    alg_bytes_step = sum(v["bytes"] for v in stats.values()) / args.steps
    # the committed traffic profile is the one of this workload with every pass boundary kept
    roof = roofline(stats, args.precision, args.steps, gp,
                    with_traffic=(n, L, ns) == (20, 20, 256) and args.ckpt == 0 and args.precision == "c64")

    out = {
        "metric": "HVPs/sec (n=20, L=20, N_s=256)",
        "value": round(hvps, 4),
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64acc" if args.precision == "c64" else "c128",
        "data": "synthetic (Haar gates, Haar brickwall U_ref of depth 2L, Haar product samples, tangent V)",
        "config": {"workload": f"brickwall HS-test HVP n={n} L={L} K={K} N_s={ns} L_ref={prob.L_ref}",
                   "precision": args.precision, "ckpt_every_layers": args.ckpt,
                   "passes_per_sweep": gp.info()["n_passes"]},
        "effective_alg_GBps": round(alg_bytes_step * hvps / 1e9, 1),
        "alg_bytes_per_hvp": alg_bytes_step,
        "setup_s": round(setup_s, 3),
        "peak_hbm_GiB": round(peak_mem / 2 ** 30, 2),
        "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in stats.items()},
        "roofline": roof,
        "targets": {"hbm_frac_target": 0.6, "met": False,
                    "note": "the north-star target of 60 % of peak HBM is not met: with passes of up to 6 "
                            "gates the backward kernel is bound by the matrix cores, not by HBM "
                            "(see roofline.compute_frac and hbm_frac)"},
    }
    if args.fixed_g_dirs > 0:
        out["fixed_G"] = fixed_g_leg(gp, prob.G, args.fixed_g_dirs, rng, hvps)
    gp.close()
    del gp
    torch.cuda.empty_cache()

    # the oracle on samples 0..3 (single-threaded processes), running while the GPU legs run
    oracle = None if pool is None else start_oracle(pool, n, L, ns, args.seed)

    if not args.no_legs:
        # accuracy references on the GPU at (prob.G, prob.V): complex64 at the headline setting
        acc_gpu = {"c64_full": one_hvp(prob, "c64", 0 if args.precision == "c64" else args.ckpt)}
        acc_gpu["c64_4"] = one_hvp(prob, "c64", 0, ns=ORACLE_SAMPLES)
        acc_gpu["c128_4"] = one_hvp(prob, "c128", 0, ns=ORACLE_SAMPLES)
        out["ckpt4"] = leg(prob, "c64", 4, 5, args.seed + 2000)
        out["ti"] = ti_leg(prob, 5, args.seed + 4000, hvps)
        out["rebuild"] = leg(prob, "c64", "rebuild", 5, args.seed + 6000)
        ck128 = pick_ckpt(n, L, prob.L_ref, ns, "c128")
        out["c128"] = leg(prob, "c128", ck128, 4, args.seed + 3000)
        acc_gpu["c128_full"] = one_hvp(prob, "c128", ck128)
        out["accuracy"] = {"c64_vs_c128_all_samples": errors(acc_gpu["c64_full"], acc_gpu["c128_full"]),
                           "c64_rebuild_vs_c128_all_samples": errors(one_hvp(prob, "c64", "rebuild"),
                                                                     acc_gpu["c128_full"])}
        c2_gpu, c2_res = c2_gpu_leg(args.seed)
        out["c2"] = {"workload": f"brickwall HS-test HVP n={C2[0]} L={C2[1]} N_s={C2[2]} L_ref={2 * C2[1]}",
                     "gpu": c2_gpu}
    if not args.no_serving:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        out["serving"] = serving_sweep(args.serve_requests, rates, args.seed)
        at1 = min(out["serving"]["rates"], key=lambda r: abs(r["rate_factor"] - 1.0))
        out["served_p50_s"] = at1["batched"]["p50_s"]
        out["served_p99_s"] = at1["batched"]["p99_s"]
    if oracle is not None:
        pool, res = oracle
        runs = res.get()
        pool.close()
        pool.join()
        t_sample = max(r[0] for r in runs)
        model, blas = cpu_info()
        P = min(MAX_HOST_WORKERS, len(os.sched_getaffinity(0)))
        out["cpu_baseline"] = {
            "value": ORACLE_SAMPLES / (ns * t_sample), "unit": "HVP/s", "cores": ORACLE_SAMPLES, "kind": "oracle",
            "sample": f"samples 0-{ORACLE_SAMPLES - 1} of the {ns} (n={n}, L={L}, K={K}) through the numpy complex128 "
                      f"oracle, one single-threaded process per sample, run together: {t_sample:.1f} s each "
                      f"(slowest); value = {ORACLE_SAMPLES} / ({ns} * t), samples are independent",
            "extrapolated_all_cores": {"cores": P, "value": P / (ns * t_sample)},
            "cpu_model": model, "blas": blas}
        if not args.no_legs:
            ref = (float(np.mean([r[1] for r in runs])), np.mean([r[2] for r in runs], axis=0),
                   np.mean([r[3] for r in runs], axis=0))
            out["accuracy"]["oracle_first_4_samples"] = {"c64": errors(acc_gpu["c64_4"], ref),
                                                         "c128": errors(acc_gpu["c128_4"], ref)}
    if c2_cpu is not None:
        # after every GPU leg and the concurrent oracle samples, so that nothing else competes for the cores
        P, wall, ref = c2_oracle_run(c2_cpu)
        c2 = out.setdefault("c2", {"workload": f"brickwall HS-test HVP n={C2[0]} L={C2[1]} N_s={C2[2]} L_ref={2 * C2[1]}"})
        c2["cpu_oracle"] = {"value": round(1.0 / wall, 4), "unit": "HVP/s", "cores": P, "kind": "oracle",
                            "measured": f"directly: all {C2[2]} samples over {P} single-threaded processes "
                                        f"(samples r, r+{P}, ... on process r), {wall:.2f} s from the first "
                                        f"process's start of the evaluation to the last one's end, labels excluded"}
        if "gpu" in c2:
            c2["accuracy_vs_oracle_all_samples"] = {prec: errors(c2_res[prec], ref) for prec in ("c64", "c128")}
            c2["gpu_vs_cpu"] = {prec: round(c2["gpu"][prec]["value"] * wall, 1) for prec in ("c64", "c128")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
