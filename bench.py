#!/usr/bin/env python3
"""Benchmark of the ReLU-QP hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a random linear MPC problem,
nx = 120 states, nu = 40 controls, horizon N = 40, condensed with LQR preconditioning into a
dense QP with n = 1600 controls and m = 1600 control limits; FP32 iteration with FP64
residuals; 8 log-spaced penalties 1e-3..1e3; sigma 1e-6, alpha 1.6, eps_abs = eps_rel = 1e-3,
max 4000 iterations, check every 25. Synthetic, seeded inputs (no dataset).

One step = one QP solve of the whole online path: the update of q, l, u from a new initial
state x0, then all iterations, residual checks and penalty switches until eps = 1e-3. Steps run
in persistent launches of at most --chunk solves each (relu_qp_solve_sequence: every solve reads
its own x0 and writes its own results; the layer weights stay on chip between the solves of a
launch); the last launch of the warm-up and of the timed region holds the remainder. The x0 of
every step are resident in HBM before the timed region starts. A separate probe times one solve
per launch (relu_qp_solve_x0) for the per-solve latency.

Prints one JSON line. `roofline` covers the persistent layer kernel: algorithmic bytes per
launch = sum over its solves of (iterations + checks) * (n^2 + 2 m n) * 4 B, over its average
launch duration from HIP events recorded on the solve stream around each launch in the timed
region. The weights stay on chip, so this is an effective rate; `roofline.traffic` is the
HBM rate the rocprofv3 counters saw for the same kernel sources (named file, else null).

With the headline workload the same line carries, under `variants`: the same family with
x0 scaled by 20 (limits bind, penalties switch), the batched matrix-core engine on 4096
instances of the family in BF16x3 and in FP32, and a short served-vs-plain latency run over the
four serving families.
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
MFMA_PEAK_TFLOPS = {"bf16x3": 2500.0, "fp32": 157.3}  # dense bf16 / fp32 matrix-core peaks
METRIC = "QP solves/sec + ADMM iters/sec at eps=1e-3; p50/p99 solve latency, served vs plain"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--x0-scale", type=float, default=1.0, help="x0 ~ scale * U[-1,1]^nx (1 = the workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--steady-iters", type=int, default=4000, help="iterations of the fixed-iteration probe")
    ap.add_argument("--chunk", type=int, default=100,
                    help="solves per persistent launch (the last launch holds the remainder)")
    ap.add_argument("--no-variants", action="store_true",
                    help="c1: leave out the x0 x 20, batched and served-vs-plain sub-records")
    ap.add_argument("--variant-steps", type=int, default=10, help="batched variants: timed steps (4096 solves each)")
    ap.add_argument("--variant-rates", default="300,3000", help="served-vs-plain variant: request rates per second")
    ap.add_argument("--variant-duration", type=float, default=2.0, help="served-vs-plain variant: seconds per rate")
    ap.add_argument("--grid", type=int, default=0, help="c0/c1/c2: workgroups per launch (0 = the library's choice)")
    ap.add_argument("--grid-sweep", default=None,
                    help="c0/c1/c2: workgroup counts for extra fixed-iteration probes (default: c0 1,2,5,10,20,40)")
    ap.add_argument("--latency-solves", type=int, default=300, help="one-solve launches timed for latency")
    ap.add_argument("--form-iters", type=int, default=2000, help="forms: layers per timed run")
    ap.add_argument("--closed-nu", default="10,40,50", help="closed: control dimensions")
    ap.add_argument("--budgets", default="1,2,15", help="closed: ADMM iterations per MPC step")
    ap.add_argument("--closed-steps", type=int, default=1000, help="closed: MPC steps per launch")
    ap.add_argument("--closed-reps", type=int, default=3)
    ap.add_argument("--x0-scale-closed", type=float, default=20.0)
    ap.add_argument("--dense-problems", type=int, default=10, help="dense: problems per size")
    ap.add_argument("--dense-reps", type=int, default=3, help="dense: timed solves per problem")
    ap.add_argument("--dense-precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only one device copy of 256 MiB (the reference for the HBM byte counters) and exit")
    ap.add_argument("--workload", choices=["c0", "c1", "c2", "batch", "serve", "dense", "closed", "forms"],
                    default="c1",
                    help="c1: one instance per solve (the headline, n = m = 1600); c0: the n = m = 20 FP64 "
                         "instance with a fixed penalty 0.1 (latency-bound); c2: one instance per solve "
                         "of the n = 600, m = 1800 family; batch: 4096 instances of the c1 family per solve on "
                         "the matrix cores; serve: continuous batching of MPC requests; dense: random dense QPs "
                         "with equality rows to eps 1e-6; closed: closed-loop MPC, fixed iterations per step; forms: compact vs the "
                         "paper's literal layer")
    ap.add_argument("--precision", choices=["bf16x3", "fp32"], default="bf16x3", help="batched engine precision")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--rates", default="100,300,1000,3000,10000,20000", help="serve: request rates per second")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals per rate")
    ap.add_argument("--slots", type=int, default=256, help="serve: slots per family")
    ap.add_argument("--families", default="f200,f800,f1600,f3200")
    ap.add_argument("--hbm-budget-gib", type=float, default=0.0,
                    help="serve: device memory the families' handles may hold together (0 = all resident)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join("profiles", "layer_kernel_c1_n1600_traffic.json")


def measured_traffic(iters_per_solve, solves_per_launch):
    """HBM bytes per launch of the layer kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the counters read for a plain copy),
    and where they came from; (None, reason) when the kernel sources changed since the counters
    were taken or no record has this launch shape (solves per launch, iterations per solve)."""
    import hashlib

    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None, "no counter record"
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest()[:16] != rec["source_sha256_16"]:
        return None, f"{TRAFFIC_FILE}: kernel sources changed since the counters were taken"
    for d in rec["dispatches"]:
        if abs(iters_per_solve - d["iterations_per_solve"]) <= 1e-9 and solves_per_launch == d["solves_per_dispatch"]:
            b = (d["fetch_kib_per_dispatch"] * rec["fetch_factor"] + d["write_kib_per_dispatch"] * rec["write_factor"])
            return b * 1024, f"{TRAFFIC_FILE} (sources sha256 {rec['source_sha256_16']}, rocprofv3 --pmc)"
    return None, f"{TRAFFIC_FILE}: no record for {solves_per_launch} solves per launch"


def _oracle_stream(prob, x0s, budget_s, n_rho=8):
    """Solves of the x0 stream by the FP64 oracle (explicit-inverse layer form, same settings)
    until the budget is spent; the offline stage (the factorisation) runs first, untimed.
    Returns (solves, ADMM iterations, seconds)."""
    import oracle
    from oracle import admm

    s = admm.Settings(n_rho=n_rho)
    cache = {}
    q, l, u = prob.instance(x0s[0])
    oracle.solve(prob.P, q, prob.A, l, u, s, cache=cache)  # offline stage, not timed
    t0 = time.perf_counter()
    done = iters = 0
    while done < len(x0s):
        q, l, u = prob.instance(x0s[done])
        iters += oracle.solve(prob.P, q, prob.A, l, u, s, cache=cache).iterations
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done, iters, time.perf_counter() - t0


def cpu_baseline(prob, x0s, budget_s, n_rho=8):
    """The FP64 oracle on the host cores: the solve stream with the BLAS threads it has (the
    reported value), then the same with BLAS on one thread."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits

        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threadpool_limits, cores = None, os.cpu_count()
    done, iters, dt = _oracle_stream(prob, x0s, budget_s / 2, n_rho)
    out = {
        "value": done / dt,
        "unit": "solves/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"first {done} solves of the same x0 stream (FP64 NumPy, {iters} ADMM iterations, "
                  f"{iters / dt:.0f} iters/s), offline stage excluded",
        "host": host_cpu(),
    }
    if threadpool_limits is not None:
        with threadpool_limits(limits=1, user_api="blas"):
            d1, i1, t1 = _oracle_stream(prob, x0s, budget_s / 2, n_rho)
        out["single_thread"] = {"value": d1 / t1, "cores": 1, "sample": f"first {d1} solves, BLAS on one thread"}
    return out


def host_cpu():
    """The host the CPU baseline ran on: CPU model, logical CPUs, and the CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = None
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


_POOL_BARRIER = None


def _pool_init(barrier):
    global _POOL_BARRIER
    _POOL_BARRIER = barrier


def _pool_solve(job):
    """One worker of the pooled baseline: its own problem copy and offline stage, then (after
    every worker is ready) its share of the x0 stream."""
    name, x0s, budget_s = job
    import oracle
    from oracle import admm
    from workloads import make_config

    prob = make_config(name)
    s = admm.Settings(n_rho=8)
    cache = {}
    q, l, u = prob.instance(x0s[0])
    oracle.solve(prob.P, q, prob.A, l, u, s, cache=cache)  # offline stage, not timed
    _POOL_BARRIER.wait()
    t0 = time.perf_counter()
    done = iters = 0
    while done < len(x0s):
        q, l, u = prob.instance(x0s[done])
        iters += oracle.solve(prob.P, q, prob.A, l, u, s, cache=cache).iterations
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done, iters, time.perf_counter() - t0


def cpu_baseline_pool(name, x0s, budget_s, workers=None):
    """The FP64 oracle on many instances: a pool of processes (one per host core, at most 16),
    each solving one instance at a time with BLAS on one thread."""
    import multiprocessing as mp

    workers = workers or min(16, os.cpu_count() or 1)
    ctx = mp.get_context("spawn")  # the workers never touch the GPU
    keys = ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        barrier = ctx.Barrier(workers)
        jobs = [(name, c, budget_s) for c in np.array_split(x0s, workers)]
        with ctx.Pool(workers, initializer=_pool_init, initargs=(barrier,)) as pool:
            res = pool.map(_pool_solve, jobs)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    done, iters, dt = sum(r[0] for r in res), sum(r[1] for r in res), max(r[2] for r in res)
    return {
        "value": done / dt,
        "unit": "solves/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{workers} processes, one instance at a time each, BLAS on one thread: {done} solves of the same "
                  f"x0 stream ({iters} ADMM iterations), offline stage excluded",
        "host": host_cpu(),
    }


def plan_launches(count: int, chunk: int) -> list:
    """Sizes of the persistent launches that run `count` solves, at most `chunk` each (the last
    holds the remainder); empty for count 0."""
    if count < 0 or chunk < 1:
        raise ValueError("count must be >= 0 and chunk >= 1")
    return [min(chunk, count - s) for s in range(0, count, chunk)]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration()
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")
    if args.workload == "batch":
        out = bench_batch(args, args.steps, args.warmup, args.precision, args.x0_scale, not args.no_cpu_baseline)
    elif args.workload == "serve":
        out = bench_serve(args, args.rates, args.duration, args.slots)
    elif args.workload == "dense":
        return bench_dense(args)
    elif args.workload == "closed":
        return bench_closed(args)
    elif args.workload == "forms":
        return bench_forms(args)
    else:
        out = bench_single(args, args.workload, args.x0_scale, args.steps, args.warmup, probes=True)
        if args.workload == "c1" and not args.no_variants:
            out["variants"] = variants(args)
    import paper_2311_18056_amd as rq

    rq.close_all()  # every handle is closed before the interpreter (and a profiler) shuts down
    print(json.dumps(out), flush=True)


def copy_calibration():
    """One device-to-device copy of 256 MiB: what rocprofv3's FETCH_SIZE and WRITE_SIZE read for
    it, against the 256 MiB each way the copy moves, gives the factors that turn the counters of a
    kernel into HBM bytes."""
    import torch

    a = torch.ones(64 * 2**20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 4}), flush=True)


def variants(args):
    """Sub-records of the headline line, each with its own workload: limits binding (x0 x 20),
    the batched engine on 4096 instances (BF16x3 and FP32), served vs plain latency."""
    v = {}
    print("variant: c1, x0 x 20", file=sys.stderr, flush=True)
    v["c1_x0x20"] = bench_single(args, "c1", 20.0, min(args.steps, 500), min(args.warmup, 50), probes=False,
                                 latency_solves=100)
    for prec in ("bf16x3", "fp32"):
        print(f"variant: batched, {prec}", file=sys.stderr, flush=True)
        v[f"batched_{prec}"] = bench_batch(args, args.variant_steps, 2, prec, 1.0, False, steady_iters=0)
    bf, fp = v["batched_bf16x3"], v["batched_fp32"]
    v["batched_bf16x3_over_fp32"] = bf["value"] / fp["value"]
    print("variant: served vs plain", file=sys.stderr, flush=True)
    v["served_vs_plain"] = bench_serve(args, args.variant_rates, args.variant_duration, 128)
    return v


def bench_single(args, workload, x0_scale, steps, warmup, probes=True, latency_solves=None):
    """One instance per solve (c0, c1, c2): `steps` timed solves of a fresh x0 each, in
    persistent sequence launches; returns the JSON record."""
    import torch

    import paper_2311_18056_amd as rq
    from workloads import make_config, x0_batch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = make_config(workload)
    n, m, nx = prob.n, prob.m, prob.nx
    total = warmup + steps
    x0_host = x0_batch(nx, total, 1000, scale=x0_scale)
    q0, l0, u0 = prob.instance(x0_host[0])

    small = workload == "c0"  # FP64 with one fixed penalty 0.1; the others FP32 over 8
    settings = dict(precision="fp64" if small else "fp32", n_rho=1 if small else 8, rho0=0.1, sigma=1e-6,
                    alpha=1.6, eps_abs=1e-3, eps_rel=1e-3, max_iter=4000, check_interval=25)
    esize = 8 if small else 4
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    sol = rq.Solver(prob.P, q0, prob.A, l0, u0, **settings)
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    if args.grid:
        sol.set_launch(args.grid)
    grid_wg, block = sol.launch()

    x0_dev = torch.tensor(x0_host, dtype=torch.float64, device=dev)  # resident before timing
    stream = torch.cuda.current_stream()
    sizes_w, sizes_t = plan_launches(warmup, args.chunk), plan_launches(steps, args.chunk)
    sizes = sizes_w + sizes_t
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    nl, nw = len(sizes), len(sizes_w)
    outs = [sol.sequence_slots(c) for c in sizes]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(nl)]
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(nl)]

    def launch(c):
        ev1[c].record(stream)
        sol.solve_sequence(x0_dev[starts[c]:starts[c + 1]], stream, out=outs[c])
        ev2[c].record(stream)

    for c in range(nw):
        launch(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(nw, nl):
        launch(c)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    it = torch.cat([o["iterations"] for o in outs[nw:]]).cpu().numpy().astype(np.int64)
    st = torch.cat([o["status"] for o in outs[nw:]]).cpu().numpy()
    kern_ms = np.array([ev1[c].elapsed_time(ev2[c]) for c in range(nw, nl)])
    solves_per_s = steps / wall
    checks = -(-it // 25)
    bytes_per_unit = (n * n + 2 * m * n) * esize
    alg_bytes = float(np.sum((it + checks) * bytes_per_unit))
    achieved_gbs = alg_bytes / (np.sum(kern_ms) * 1e-3) / 1e9

    # per-solve latency: one solve per launch, arrival of x0 (in HBM) to results written
    lat_ms = []
    n_lat = args.latency_solves if latency_solves is None else latency_solves
    if n_lat > 0:
        slots1, res1 = sol.result_slots(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for i in range(n_lat + 10):
            e0.record(stream)
            sol.solve_x0(x0_dev[i % total], stream, out=res1[0])
            e1.record(stream)
            e1.synchronize()
            if i >= 10:
                lat_ms.append(e0.elapsed_time(e1))
    step_ms = np.array(lat_ms) if lat_ms else np.array([np.nan])

    # fixed-iteration probe: per-iteration time of the same kernel without the stopping test
    def fixed_probe(grid):
        fx = rq.Solver(prob.P, q0, prob.A, l0, u0, **dict(settings, eps_abs=0.0, eps_rel=0.0,
                                                          max_iter=args.steady_iters))
        fx.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        if grid:
            fx.set_launch(grid)
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
        fx.close()
        ms = min(times)
        k = args.steady_iters
        nck = -(-k // 25)
        return {
            "iterations": k,
            "ms": ms,
            "us_per_iter": ms * 1e3 / k,
            "effective_GBs": (k + nck) * bytes_per_unit / (ms * 1e-3) / 1e9,
        }

    steady = fixed_probe(args.grid) if probes and args.steady_iters > 0 else None
    sweep_arg = args.grid_sweep if args.grid_sweep is not None else ("1,2,5,10,20,40" if small else "")
    sweep = None
    if probes and args.steady_iters > 0 and sweep_arg:
        sweep = {}
        for g in (int(v) for v in sweep_arg.split(",")):
            print(f"fixed-iteration probe at {g} workgroups", file=sys.stderr, flush=True)
            sweep[str(g)] = fixed_probe(g)["us_per_iter"] * 1e3

    cpu = None
    if probes and not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, x0_host[warmup:], args.cpu_seconds, settings["n_rho"])

    traffic_bytes, traffic_src = None, None
    if workload == "c1":
        traffic_bytes, traffic_src = measured_traffic(float(np.mean(it)), sizes_t[0] if len(set(sizes_t)) == 1 else -1)
    avg_launch_s = float(np.mean(kern_ms)) * 1e-3
    roof = {
        "bound": "hbm",
        "achieved": achieved_gbs,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved_gbs / HBM_PEAK_GBS,
        "frac_kind": "effective: algorithmic bytes of the two-GEMV form over the launch time; the weights stay "
                     "on chip, so the kernel is bound by its per-iteration exchange latency, not by HBM",
        # measured HBM bytes per launch (rocprofv3 counters) over the same launch duration
        "traffic": None if traffic_bytes is None else traffic_bytes / avg_launch_s / 1e9,
        "traffic_frac_of_peak": None if traffic_bytes is None else traffic_bytes / avg_launch_s / 1e9 / HBM_PEAK_GBS,
        "traffic_bytes_per_launch": traffic_bytes,
        "traffic_source": traffic_src,
        "kernel": ("layer_kernel<float, 4, 8, 8, false>" if workload == "c1"
                   else "small_kernel<double, 8, 8>" if small and grid_wg == 1
                   else f"layer_kernel<{'double' if small else 'float'}, ...>"),
        "alg_bytes_per_unit": bytes_per_unit,
        "avg_launch_us": float(np.mean(kern_ms) * 1e3),
        "solves_per_launch": sizes_t,
    }
    if steady:
        roof["us_per_iter_fixed"] = steady["us_per_iter"]
    if small:
        # n = m = 20: the layer weights sit in registers and an iteration is one on-chip exchange of
        # the 40-entry layer input, so its time is a latency, not a share of a bandwidth or a peak
        roof.update(bound="latency", achieved=steady["us_per_iter"] * 1e3 if steady else None, peak=None,
                    unit="ns/iteration", frac=None, hbm_equivalent_GBs=achieved_gbs)
    out = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if small else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"random linear MPC, LQR-condensed dense QP, n={n}, m={m} "
                         f"(nx={nx}, nu={prob.nu}, N={prob.N}), one instance per solve"),
            "x0": f"{x0_scale:g} * U[-1,1]^{nx}, seed 1000",
            "penalties": "fixed 0.1" if small else "8 log-spaced 1e-3..1e3",
            "eps": 1e-3,
            "step": "one solve: q, l, u from a new x0, iterations and checks to eps",
            "launch": {"grid": grid_wg, "block": block},
        },
        "admm_iters_per_s": float(np.sum(it)) / wall,
        "iters_per_solve": float(np.mean(it)),
        "status_counts": {rq.STATUS_NAMES[int(s)]: int(np.sum(st == s)) for s in np.unique(st)},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "note": "plain: one solve per launch, events around the launch"},
        "setup_ms": setup_ms,
        "steady_state": steady,
        "ns_per_iter_by_grid": sweep,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    sol.close()
    return out


def bench_batch(args, steps, warmup, precision, x0_scale, with_cpu, steady_iters=None):
    """B instances of the configuration-1 family (same P and A, x0 per instance) per solve on
    the batched matrix-core engine. One step = device update of every instance's q, l, u plus
    one persistent solve of all of them to eps = 1e-3. Returns the JSON record."""
    import torch

    import paper_2311_18056_amd as rq
    from workloads import make_config, x0_batch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = make_config("c1")
    n, m, nx, B = prob.n, prob.m, prob.nx, args.batch
    total = steps + warmup
    steady_iters = args.steady_iters if steady_iters is None else steady_iters
    # instance i of step s: x0 from seed 3_000_000 + s (B rows)
    x0_host = np.stack([x0_batch(nx, B, 3_000_000 + s, scale=x0_scale) for s in range(total)])
    q0, l0, u0 = prob.instance(x0_host[0])
    settings = dict(precision=precision, engine="batch", n_rho=8, sigma=1e-6, alpha=1.6, eps_abs=1e-3,
                    eps_rel=1e-3, max_iter=4000, check_interval=25)
    t_setup = time.perf_counter()
    sol = rq.Solver(prob.P, q0, prob.A, l0, u0, **settings)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    x0_dev = torch.tensor(x0_host, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(total)]
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(total)]
    its, sts = [], []

    def step(i):
        sol.update_x0_device(x0_dev[i], stream)
        ev1[i].record(stream)
        sol.solve(stream)
        ev2[i].record(stream)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, total):
        step(i)
        # results are overwritten by the next solve: keep counts on the device stream
        its.append(sol.iterations.clone())
        sts.append(sol.status.clone())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    it = torch.stack(its).cpu().numpy().astype(np.int64)
    st = torch.stack(sts).cpu().numpy()
    kern_ms = np.array([ev1[i].elapsed_time(ev2[i]) for i in range(warmup, total)])
    checks = -(-it // 25)
    flops_per_unit = 2.0 * (n * n + 2 * m * n)  # useful flops per instance-iteration
    alg_flops = float(np.sum((it + checks) * flops_per_unit))
    achieved = alg_flops / (np.sum(kern_ms) * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[precision]

    steady = None
    if steady_iters > 0:
        k = min(steady_iters, 200)
        fx = rq.Solver(prob.P, q0, prob.A, l0, u0, **dict(settings, eps_abs=0.0, eps_rel=0.0, max_iter=k))
        fx.set_tile(sol.tile()[0])  # the shape the timed solves ran with
        fx.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        fx.update_x0_device(x0_dev[0], stream)
        fx.solve(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fx.solve(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        nck = -(-k // 25)
        steady = {"iterations": k, "ms": ms, "us_per_iter": ms * 1e3 / k,
                  "useful_TFLOPs": B * (k + nck) * flops_per_unit / (ms * 1e-3) / 1e12}
        fx.close()

    out = {
        "metric": METRIC,
        "value": B * steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if precision == "bf16x3" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{B} instances per solve of the n=1600, m=1600 MPC family (nx=120, nu=40, N=40), "
                        "batched matrix-core engine",
            "x0": f"{x0_scale:g} * U[-1,1]^120, seed 3000000 + step",
            "penalties": "8 log-spaced 1e-3..1e3",
            "eps": 1e-3,
            "step": f"q, l, u of {B} instances from new x0, one persistent solve of all of them to eps",
        },
        "admm_iters_per_s": float(np.sum(it)) / wall,
        "iters_per_solve": float(np.mean(it)),
        "status_counts": {rq.STATUS_NAMES[int(s)]: int(np.sum(st == s)) for s in np.unique(st)},
        "latency_ms": {"p50": float(np.percentile(kern_ms, 50)), "p99": float(np.percentile(kern_ms, 99)),
                       "note": "every instance of a step completes with its launch: the launch duration (events)"},
        "setup_ms": setup_ms,
        "tile_autotuner": {"rows": sol.tile()[0], "us_per_iter": sol.tile()[1]},
        "steady_state": steady,
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "kernel": f"batch_kernel<{1 if precision == 'bf16x3' else 0}, {sol.tile()[0]}>",
            "alg_flops_per_unit": flops_per_unit,
            "avg_launch_us": float(np.mean(kern_ms) * 1e3),
        },
        "cpu_baseline": cpu_baseline_pool("c1", x0_host[warmup:].reshape(-1, nx), args.cpu_seconds) if with_cpu
        else None,
    }
    sol.close()
    return out


def dense_sizes(count: int = 10):
    """n log-spaced from 10 to 2000 (Sec. V-A), rounded to multiples of 4 above 10."""
    return [10] + [int(round(v / 4.0)) * 4 for v in np.logspace(1, np.log10(2000), count)[1:]]


def bench_dense(args):
    """Random dense QPs with n/4 equality and n/4 inequality rows (Sec. V-A): for each size,
    ``--dense-problems`` problems, each solved ``--dense-reps`` times from a cold start to
    residuals below eps_abs = eps_rel = 1e-6 (equality rows at 1e3 times the penalty, 8 penalties).
    Solve time = the persistent launch (HIP events), problem data resident; setup reported apart."""
    import torch

    import paper_2311_18056_amd as rq
    from workloads import random_qp

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    settings = dict(precision=args.dense_precision, n_rho=8, sigma=1e-6, alpha=1.6, eps_abs=1e-6, eps_rel=1e-6,
                    max_iter=20000, check_interval=25)
    rows = []
    es = 8 if args.dense_precision == "fp64" else 4
    for n in dense_sizes():
        me = mi = n // 4
        ms_all, its, sts, setup = [], [], [], []
        for k in range(args.dense_problems):
            P, q, A, l, u = random_qp(n, me, mi, seed=10_000 * n + k)
            t0 = time.perf_counter()
            sol = rq.Solver(P, q, A, l, u, **settings)
            setup.append((time.perf_counter() - t0) * 1e3)
            sol.solve(stream)  # warm-up (kernel load, weights to L2)
            for _ in range(args.dense_reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sol.solve(stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms_all.append(e0.elapsed_time(e1))
            r = sol.result()
            its.append(int(r["iterations"]))
            sts.append(int(r["status"]))
            sol.close()
        m = me + mi
        it = np.array(its)
        ms = float(np.mean(ms_all))
        bytes_iter = (n * n + 2 * m * n) * es
        rows.append({"n": n, "m_eq": me, "m_ineq": mi, "solve_ms_mean": ms, "solve_ms_median": float(np.median(ms_all)),
                     "iterations_mean": float(it.mean()), "iterations_max": int(it.max()),
                     "solved": int(sum(1 for x in sts if x == rq.RQP_SOLVED)), "problems": len(sts),
                     "setup_ms_mean": float(np.mean(setup)),
                     "effective_GBs": float((it.mean() + np.ceil(it.mean() / 25)) * bytes_iter / (ms * 1e-3) / 1e9)})
        print(json.dumps(rows[-1]), flush=True)
    big = rows[-1]
    paper_s = 1.62e-2  # the paper's solve time at n = 2000 (Fig. 2; RTX 3080, precision not stated)
    out = {
        "metric": "random dense QP solve time to eps 1e-6 (Sec. V-A sizes)",
        "value": 1e3 / big["solve_ms_mean"],
        "unit": "solves/s at n=2000",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": (1e3 / big["solve_ms_mean"]) / (1.0 / paper_s),
        "baseline": {"value": 1.0 / paper_s, "source": "paper Fig. 2, n = 2000, RTX 3080 (context, other hardware)"},
        "dtype": "f64" if args.dense_precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "random dense QPs, n log-spaced 10..2000, n/4 equality + n/4 inequality rows, "
                               "eps_abs = eps_rel = 1e-6, 8 penalties, cold starts",
                   "problems_per_size": args.dense_problems, "reps": args.dense_reps},
        "sizes": rows,
        "roofline": {"bound": "hbm", "achieved": big["effective_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": big["effective_GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"layer_kernel ({args.dense_precision}), n = 2000",
                     "alg_bytes_per_unit": (2000 * 2000 + 2 * 1000 * 2000) * es},
        "cpu_baseline": None if args.no_cpu_baseline else dense_cpu_baseline(settings, args.cpu_seconds),
    }
    print(json.dumps(out), flush=True)


def dense_cpu_baseline(settings, budget_s):
    """The FP64 oracle on the same problems (largest size first), offline stage excluded."""
    import oracle
    from oracle import admm
    from workloads import random_qp

    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    s = admm.Settings(n_rho=8, eps_abs=settings["eps_abs"], eps_rel=settings["eps_rel"], max_iter=settings["max_iter"])
    n = dense_sizes()[-1]
    done, dt = 0, 0.0
    while dt < budget_s and done < 10:
        P, q, A, l, u = random_qp(n, n // 4, n // 4, seed=10_000 * n + done)
        cache = {}
        oracle.solve(P, q, A, l, u, s, cache=cache)  # offline stage, not timed
        t0 = time.perf_counter()
        oracle.solve(P, q, A, l, u, s, cache=cache)
        dt += time.perf_counter() - t0
        done += 1
    return {"value": done / dt, "unit": "solves/s at n=2000", "cores": int(cores), "kind": "oracle",
            "sample": f"{done} of the n = 2000 problems, each solved once to 1e-6 after an untimed setup",
            "host": host_cpu()}


def bench_forms(args):
    """Layer forms at alpha = 1 and a fixed penalty (0.1), FP32: the compact form the solver runs
    ([x; z] rows, (n+m)^2 weights held on chip) against the paper's literal layer ([x; z; lambda]
    rows, (n+2m)^2 weights streamed every layer), both one exchange per layer. Fixed iteration
    counts; the compact run checks once at the end."""
    import torch

    import paper_2311_18056_amd as rq
    from workloads import make_config, x0_batch

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    K = args.form_iters
    rows = []
    for name, scale in (("c1", 20.0), ("c2", 3.0)):
        prob = make_config(name)
        q, l, u = prob.instance(scale * x0_batch(prob.nx, 1, 1001)[0])
        n, m = prob.n, prob.m
        sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp32", alpha=1.0, n_rho=1, rho0=0.1, eps_abs=0.0,
                        eps_rel=0.0, max_iter=K, check_interval=K)
        res = {}
        for form, run in (("compact", lambda: sol.solve(stream)), ("paper", lambda: sol.solve_paper_form(K, stream))):
            run()  # warm-up (and the paper form's one-time weight build)
            torch.cuda.synchronize()
            ms = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                run()
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            res[form] = float(np.min(ms)) * 1e3 / K
        rows.append({"workload": name, "n": n, "m": m, "iterations": K,
                     "compact_us_per_iter": res["compact"], "paper_us_per_iter": res["paper"],
                     "compact_weight_MB": (n + m) ** 2 * 4 / 1e6, "paper_weight_MB": (n + 2 * m) ** 2 * 4 / 1e6,
                     "paper_streamed_TBs": (n + 2 * m) ** 2 * 4 / (res["paper"] * 1e-6) / 1e12})
        print(json.dumps(rows[-1]), flush=True)
        sol.close()
    print(json.dumps({"metric": "us per layer, compact vs the paper's literal layer (alpha 1, fixed penalty)",
                      "unit": "us", "n_gpus": 1, "dtype": "f32", "data": "synthetic", "runs": rows}), flush=True)


# MPC step times the paper reports for one ADMM iteration per step (Fig. 1, RTX 3080; context)
PAPER_MPC_STEP_S = {10: 1.204e-4, 50: 7.376e-4}


def bench_closed(args):
    """Closed-loop MPC of random linear systems (Sec. V-B): nu controls, nx = 3 nu states,
    horizon 40, control limits, LQR-preconditioned condensing; x0 = scale * U[-1,1]^nx. Each
    launch runs --closed-steps MPC steps (relu_qp_closed_loop: update, --budget warm-started
    iterations, applied control, plant step, all on the device); time per MPC step = launch time
    (HIP events) / steps."""
    import torch

    import paper_2311_18056_amd as rq
    from workloads import random_mpc, x0_batch

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rows = []
    for nu in [int(v) for v in args.closed_nu.split(",")]:
        prob = random_mpc(3 * nu, nu, 40, seed=60 + nu, radius=1.05, q_kind="identity", r_scale=0.1)
        x0 = args.x0_scale_closed * x0_batch(prob.nx, 1, 70 + nu)[0]
        q, l, u = prob.instance(x0)
        for budget in [int(b) for b in args.budgets.split(",")]:
            sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp32", engine="single", n_rho=8, eps_abs=0.0,
                            eps_rel=0.0, max_iter=budget)
            sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
            T = args.closed_steps
            xd = torch.tensor(x0, dtype=torch.float64, device="cuda")
            Ad = torch.tensor(prob.A_dyn, dtype=torch.float64, device="cuda")
            Bd = torch.tensor(prob.B, dtype=torch.float64, device="cuda")
            out = sol.closed_loop(xd, T, Ad, Bd, nu, stream)  # warm-up launch
            torch.cuda.synchronize()
            ms = []
            for _ in range(args.closed_reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sol.closed_loop(xd, T, Ad, Bd, nu, stream, out=out)
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            us_ = out["traj_u"].cpu().numpy()
            xs_ = out["traj_x"].cpu().numpy()
            step_s = float(np.mean(ms)) * 1e-3 / T
            row = {"nu": nu, "nx": prob.nx, "n": prob.n, "m": prob.m, "budget": budget, "steps": T,
                   "step_us": step_s * 1e6, "steps_per_s": 1.0 / step_s,
                   "active_frac": float(np.mean(np.max(np.abs(us_), axis=1) > 0.999)),
                   "x_norm_first_last": [float(np.max(np.abs(xs_[0]))), float(np.max(np.abs(xs_[-1])))]}
            if budget == 1 and nu in PAPER_MPC_STEP_S:
                row["paper_step_us"] = PAPER_MPC_STEP_S[nu] * 1e6
                row["vs_paper"] = PAPER_MPC_STEP_S[nu] / step_s
            rows.append(row)
            print(json.dumps(row), flush=True)
            sol.close()
    head = next((r for r in rows if r["nu"] == 50 and r["budget"] == 1), rows[-1])
    out = {
        "metric": "closed-loop MPC step time, one warm-started ADMM iteration per step (Fig. 1 workload)",
        "value": head["steps_per_s"],
        "unit": f"MPC steps/s at nu={head['nu']}, budget {head['budget']}",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": head.get("vs_paper"),
        "baseline": {"value_s": PAPER_MPC_STEP_S.get(head["nu"]), "source": "paper Fig. 1, RTX 3080 (context)"},
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "random linear MPC closed loop, nx = 3 nu, N = 40, control limits, LQR-condensed, "
                               f"x0 = {args.x0_scale_closed:g} * U[-1,1]^nx, plant = model",
                   "steps_per_launch": args.closed_steps},
        "runs": rows,
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, rates, duration, slots):
    """Open-loop Poisson requests over four MPC families, served by continuous batching vs one
    at a time on the single-instance engine; p50/p99 latency per offered rate. Returns the
    JSON record."""
    import torch

    from paper_2311_18056_amd import Solver
    from paper_2311_18056_amd.serving import Family, Server, latency_summary, poisson_requests, serve_plain
    from workloads import make_config

    torch.cuda.set_device(0)
    probs = [make_config(f) for f in args.families.split(",")]
    gens = [lambda rng, p=p: args.x0_scale * rng.uniform(-1.0, 1.0, p.nx) for p in probs]
    settings = dict(n_rho=8, sigma=1e-6, alpha=1.6, eps_abs=1e-3, eps_rel=1e-3, max_iter=4000, check_interval=25)
    budget = int(args.hbm_budget_gib * 2**30) if args.hbm_budget_gib > 0 else None
    fams = [Family.from_mpc(p, slots=slots, precision=args.precision, lazy=budget is not None,
                            **settings).attach_single(p, **settings) for p in probs]
    singles = []
    for p in probs:
        q, l, u = p.instance(np.zeros(p.nx))
        s = Solver(p.P, q, p.A, l, u, precision="fp32", **settings)
        s.set_parametric(p.F, p.E, p.lo, p.hi)
        singles.append(s)
    rows = []
    for i, rate in enumerate(float(r) for r in rates.split(",")):
        count = int(min(20000, rate * duration))
        reqs = poisson_requests(rate, count, duration, gens, seed=4 + i)
        for f in fams:
            f.pin = None
        warm_s = 0.1 * max(r.t_arrival for r in reqs)  # arrivals in the first 10 % are warm-up
        srv = Server(fams, n_checks=1, warm=True, hbm_budget=budget)
        srv.run(reqs, time_limit=duration * 3)
        served = latency_summary(reqs, warmup=warm_s)
        mem = srv.memory
        served["memory"] = {"budget_gib": None if budget is None else budget / 2**30,
                            "peak_resident_gib": mem.peak / 2**30, "loads": mem.loads, "evictions": mem.evictions}
        reqs = poisson_requests(rate, count, duration, gens, seed=4 + i)
        serve_plain(singles, reqs, time_limit=duration * 3)
        plain = latency_summary(reqs, warmup=warm_s)
        rows.append({"rate": rate, "served": served, "plain": plain})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    out = {
        "metric": "p50/p99 solve latency, served vs plain",
        "unit": "ms",
        "n_gpus": 1,
        "data": "synthetic",
        "config": {"workload": "MPC families " + args.families + ", Poisson arrivals, family uniform",
                   "seconds_per_rate": duration,
                   "slots_per_family": slots, "precision": args.precision, "x0_scale": args.x0_scale,
                   "family_gib": {name: f.bytes / 2**30 for name, f in zip(args.families.split(","), fams)}},
        "rates": rows,
    }
    for f in fams:
        f.close()
    for s in singles:
        s.close()
    return out


if __name__ == "__main__":
    main()
