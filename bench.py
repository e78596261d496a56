"""Benchmark: Hessian-vector products per second of the brickwall Hilbert-Schmidt cost at
n=20 qubits, L=20 layers (K=190 gates), N_s=256 Haar product samples, U_ref a Haar brickwall
of depth 40, complex64 states with FP64 accumulation, on one MI355X.

One step = one from-scratch HVP call (cost + gradient + HVP for one (G, V) over all samples),
each at its own Haar G, so that no forward state kept from an earlier call belongs to it; the
labels phi_s = U_ref psi_s are computed once per problem (the problem statement takes them as
input) and reported separately as setup time.  A second leg ("fixed_G") times HVPs along several
directions at one G, where the forward states at G are kept between calls.  Prints one JSON line.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--L", type=int, default=20)
    ap.add_argument("--ns", type=int, default=256)
    ap.add_argument("--precision", default="c64", choices=["c64", "c128"])
    ap.add_argument("--ckpt", type=int, default=None,
                    help="layer checkpoint interval (0: every pass boundary; default: the fastest that fits)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 2 GiB device copy 5 times (calibrates HBM traffic counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--fixed-g-dirs", type=int, default=8,
                    help="directions of the fixed-G leg (0: skip it)")
    ap.add_argument("--seed", type=int, default=1)
    return ap.parse_args()


def cpu_baseline(n, L, seed):
    """The oracle (numpy complex128 statevector Alg. 1 + 2) on one sample of the same workload."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import circuit, sv
    from paper_2604_20384_amd.inputs import make_problem

    p = make_problem(n, L, 1, seed=seed)
    psi, phi = circuit.labels(p.uref, p.samples, n, p.L_ref)
    t0 = time.perf_counter()
    sv.evaluate(psi, phi, p.G, p.V, n, L, batch=1)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return dt, threads


def serving(n_req, seed):
    """Poisson stream of mixed grad / HVP requests (complex64) at 0.9x the measured serial
    capacity, served one at a time (FIFO) and with continuous batching over 4 streams."""
    import numpy as np

    from paper_2604_20384_amd import serve

    rng = np.random.default_rng(seed)
    reqs = [serve.random_request(rng, n_range=(10, 20), L_range=(4, 16), ns_range=(16, 128))
            for _ in range(n_req)]
    # warm-up (first launches, allocator)
    budget = 96 << 30
    w = serve.Server(serve.GpuExecutor(), slots=1, memory_budget=budget)
    w.submit(reqs[0]).result()
    w.shutdown()
    # serial capacity: all requests queued at once, one slot
    srv = serve.Server(serve.GpuExecutor(), slots=1, memory_budget=budget)
    res, t0, t1 = serve.replay(srv, reqs, np.zeros(n_req))
    srv.shutdown()
    mu = n_req / (t1 - t0)
    lam = 0.9 * mu
    arrivals = serve.poisson_arrivals(rng, lam, n_req)
    out = {"requests": n_req, "n": [10, 20], "L": [4, 16], "N_s": [16, 128], "precision": "c64",
           "memory_budget_GiB": budget >> 30, "slots": 4,
           "serial_capacity_rps": round(mu, 3), "arrival_rate_rps": round(lam, 3)}
    for name, slots in (("serial", 1), ("batched", 4)):
        srv = serve.Server(serve.GpuExecutor(), slots=slots, memory_budget=budget)
        res, t0, t1 = serve.replay(srv, reqs, arrivals)
        srv.shutdown()
        rep = serve.latency_report(res, t0, t1)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
    return out


def measured_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_bwd_out_c64.json")
    src = os.path.join(ROOT, "paper_2604_20384_amd", "csrc", "qhvp_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel") != kernel_name or not sha.startswith(rec["kernel_source_sha256_prefix"]):
        return None
    return (rec["fetch_kib_per_launch"] * rec["fetch_factor"] + rec["write_kib_per_launch"] * rec["write_factor"]) * 1024


def copy_probe():
    import torch
    nbytes = 2 << 30
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}))


def pick_ckpt(n, L, L_ref, ns, precision):
    """Fastest checkpoint policy whose workspace fits the free HBM (8 GiB kept back)."""
    import torch

    from paper_2604_20384_amd.api import workspace_bytes
    free, _ = torch.cuda.mem_get_info()
    for ck in (0, -2, 1, 2, 4, 8):
        if workspace_bytes(n, L, L_ref, ns, precision, ck, True) <= free - (8 << 30):
            return ck
    return 8


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
    return {"directions": M, "value": round(M / dt, 4), "unit": "HVP/s", "ms_per_hvp": round(1e3 * dt / M, 3),
            "kernel_ms_per_hvp": {k: round(v["ms"] / M, 3) for k, v in stats.items()},
            "alg_bytes_per_hvp": sum(v["bytes"] for v in stats.values()) / M,
            "vs_from_scratch": round(M / dt / from_scratch_hvps, 4)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

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
    t0 = time.perf_counter()
    gp = Problem(n, L, prob.uref, prob.samples, L_ref=prob.L_ref, precision=args.precision,
                 ckpt_every=args.ckpt, device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    for i in range(args.warmup):
        gp.hvp(Gs[i], Vs[i])
    gp.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        c, g, h = gp.hvp(Gs[i], Vs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = gp.kernel_stats()
    peak_mem = torch.cuda.max_memory_allocated()
    hvps = args.steps / dt
    ms_per_step = 1e3 * dt / args.steps

    S = ns * 2 ** n * (8 if args.precision == "c64" else 16)
    alg_bytes_step = sum(v["bytes"] for v in stats.values()) / args.steps

    # dominant kernel: most device time over the timed region
    dom = max(("forward", "recompute", "backward"), key=lambda k: stats[k]["ms"])
    st = stats[dom]
    avg_ms = st["ms"] / max(1, st["launches"])
    bytes_per_launch = st["bytes"] / max(1, st["launches"])
    flops_per_launch = st["flops"] / max(1, st["launches"])
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    tfs = flops_per_launch / (avg_ms * 1e-3) / 1e12
    unit_name, comp_peak = COMPUTE_PEAK[args.precision]
    frac_hbm, frac_comp = gbs / HBM_PEAK_GBS, tfs / comp_peak
    if frac_hbm >= frac_comp:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(frac_hbm, 4)}
    else:
        roof = {"bound": unit_name, "achieved": round(tfs, 2), "peak": comp_peak, "unit": "TFLOP/s",
                "frac": round(frac_comp, 4)}
    rt = "float" if args.precision == "c64" else "double"
    bwd_name = "k_bwd_out" if gp.backward_from_outputs else "k_bwd"
    kname = f"{bwd_name}<{rt},true>" if dom == "backward" else f"k_fwd<{rt},true>"
    traffic = measured_traffic(kname) if (n, L, ns) == (20, 20, 256) else None
    roof.update({"traffic": traffic, "kernel": kname,
                 "avg_launch_ms": round(avg_ms, 4), "launches": st["launches"],
                 "alg_bytes_per_launch": bytes_per_launch, "alg_flops_per_launch": flops_per_launch,
                 "hbm_frac": round(frac_hbm, 4), "compute_frac": round(frac_comp, 4),
                 "compute_peak_TFLOPs": comp_peak})

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
    }
    if args.fixed_g_dirs > 0:
        out["fixed_G"] = fixed_g_leg(gp, prob.G, args.fixed_g_dirs, rng, hvps)
    gp.close()
    del gp
    torch.cuda.empty_cache()
    if not args.no_serving:
        out["serving"] = serving(args.serve_requests, args.seed)
        out["served_p50_s"] = out["serving"]["batched"]["p50_s"]
        out["served_p99_s"] = out["serving"]["batched"]["p99_s"]
    if not args.no_cpu_baseline:
        t_sample, threads = cpu_baseline(n, L, args.seed)
        out["cpu_baseline"] = {"value": 1.0 / (ns * t_sample), "unit": "HVP/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"one of the {ns} samples (n={n}, L={L}) through the numpy complex128 "
                                         f"oracle took {t_sample:.1f} s; value = 1 / ({ns} * t), samples are independent"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
