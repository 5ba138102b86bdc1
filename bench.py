#!/usr/bin/env python3
"""Benchmark of the ReLU-QP hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a random linear MPC problem,
nx = 120 states, nu = 40 controls, horizon N = 40, condensed with LQR preconditioning into a
dense QP with n = 1600 controls and m = 1600 control limits; FP32 iteration with FP64
residuals; 8 log-spaced penalties 1e-3..1e3; sigma 1e-6, alpha 1.6, eps_abs = eps_rel = 1e-3,
max 4000 iterations, check every 25. Synthetic, seeded inputs (no dataset).

One step = one QP solve of the whole online path: the per-solve update of q, l, u from a new
initial state x0 on the GPU, then the persistent solve kernel (all iterations, residual
checks and penalty switches) until eps = 1e-3. The x0 of every step are resident in HBM
before the timed region starts.

Prints one JSON line. `roofline` covers the persistent layer kernel: algorithmic bytes per
launch = (iterations + checks) * (n^2 + 2 m n) * 4 B, over its average launch duration from
HIP events recorded on the solve stream around each launch in the timed region.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--x0-scale", type=float, default=1.0, help="x0 ~ scale * U[-1,1]^nx (1 = the workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--steady-iters", type=int, default=2000, help="iterations of the fixed-iteration probe")
    return ap.parse_args()


def cpu_baseline(prob, x0s, budget_s):
    """The FP64 oracle (explicit-inverse layer form) on the host cores, same settings."""
    import oracle
    from oracle import admm

    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    s = admm.Settings(n_rho=8)
    cache = {}
    q, l, u = prob.instance(x0s[0])
    oracle.solve(prob.P, q, prob.A, l, u, s, cache=cache)  # offline stage, not timed
    t0 = time.perf_counter()
    done = iters = 0
    while done < len(x0s):
        q, l, u = prob.instance(x0s[done])
        r = oracle.solve(prob.P, q, prob.A, l, u, s, cache=cache)
        iters += r.iterations
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {
        "value": done / dt,
        "unit": "solves/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"first {done} solves of the same x0 stream (FP64 NumPy, {iters} ADMM iterations, "
                  f"{iters / dt:.0f} iters/s), offline stage excluded",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2311_18056_amd as rq
    from workloads import make_config, x0_batch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = make_config("c1")
    n, m, nx = prob.n, prob.m, prob.nx
    total = args.warmup + args.steps
    x0_host = x0_batch(nx, total, 1000, scale=args.x0_scale)
    q0, l0, u0 = prob.instance(x0_host[0])

    settings = dict(precision="fp32", n_rho=8, sigma=1e-6, alpha=1.6, eps_abs=1e-3, eps_rel=1e-3, max_iter=4000,
                    check_interval=25)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    sol = rq.Solver(prob.P, q0, prob.A, l0, u0, **settings)
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    grid_wg, block = sol.launch()

    x0_dev = torch.tensor(x0_host, dtype=torch.float64, device=dev)  # resident before timing
    slots, results = sol.result_slots(total)
    stream = torch.cuda.current_stream()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(total)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(total)]
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(total)]

    def step(i):
        ev0[i].record(stream)
        sol.update_x0_device(x0_dev[i], stream)
        ev1[i].record(stream)
        sol.solve(stream, out=results[i])
        ev2[i].record(stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, total):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    it = slots["iterations"][args.warmup:].cpu().numpy().astype(np.int64)
    st = slots["status"][args.warmup:].cpu().numpy()
    kern_ms = np.array([ev1[i].elapsed_time(ev2[i]) for i in range(args.warmup, total)])
    step_ms = np.array([ev0[i].elapsed_time(ev2[i]) for i in range(args.warmup, total)])
    solves_per_s = args.steps / wall
    checks = -(-it // 25)
    bytes_per_unit = (n * n + 2 * m * n) * 4
    alg_bytes = float(np.sum((it + checks) * bytes_per_unit))
    achieved_gbs = alg_bytes / (np.sum(kern_ms) * 1e-3) / 1e9

    # fixed-iteration probe: per-iteration time of the same kernel without the stopping test
    steady = None
    if args.steady_iters > 0:
        fx = rq.Solver(prob.P, q0, prob.A, l0, u0, **dict(settings, eps_abs=0.0, eps_rel=0.0,
                                                          max_iter=args.steady_iters))
        fx.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        fx.update_x0_device(x0_dev[0], stream)
        fx.solve(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(3):
            e0.record(stream)
            fx.solve(stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = min(times)
        k = args.steady_iters
        nck = -(-k // 25)
        steady = {
            "iterations": k,
            "ms": ms,
            "us_per_iter": ms * 1e3 / k,
            "effective_GBs": (k + nck) * bytes_per_unit / (ms * 1e-3) / 1e9,
        }
        fx.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, x0_host[args.warmup:], args.cpu_seconds)

    out = {
        "metric": "QP solves/sec at eps=1e-3 (with ADMM iters/sec and p50/p99 solve latency)",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "random linear MPC, LQR-condensed dense QP, n=1600, m=1600 (nx=120, nu=40, N=40)",
            "x0": f"{args.x0_scale:g} * U[-1,1]^120, seed 1000",
            "penalties": "8 log-spaced 1e-3..1e3",
            "eps": 1e-3,
            "launch": {"grid": grid_wg, "block": block},
        },
        "admm_iters_per_s": float(np.sum(it)) / wall,
        "iters_per_solve": float(np.mean(it)),
        "status_counts": {rq.STATUS_NAMES[int(s)]: int(np.sum(st == s)) for s in np.unique(st)},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "kernel_p50": float(np.percentile(kern_ms, 50))},
        "setup_ms": setup_ms,
        "steady_state": steady,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "layer_kernel<float,4,8>",
            "alg_bytes_per_unit": bytes_per_unit,
            "avg_launch_us": float(np.mean(kern_ms) * 1e3),
        },
        "cpu_baseline": cpu,
    }
    sol.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
