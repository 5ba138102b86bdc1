"""Continuous batching of MPC solve requests over QP families (host scheduling only).

A family is one QP structure (fixed P and A, so one set of device-resident layer weights)
served by a batched handle whose ``slots`` instances are request slots. Requests carry an
initial state x0 (Sec. IV: q = F x0, l = lo - E x0, u = hi - E x0). Between steps the
scheduler admits arrived requests into free slots, optionally warm-started from the family's
most recent solution shifted by one stage (the receding-horizon warm start of Sec. II-B and
Sec. V-B), runs one step (a persistent launch of ``n_checks`` check intervals) per family with
work, and retires slots whose status became final. All arithmetic runs in the HIP library.

With a single-instance handle attached (``Family.attach_single``), a family whose queue is
short and whose slots are all free is served by one sequence launch of the single-instance
engine instead (``relu_qp_solve_sequence``: the few queued requests back to back, cold starts):
at light load a batched step over a nearly empty batch of a large family costs far more than a
handful of single-instance solves.

Latency is measured from a request's arrival time to the moment its result is on the host.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from ._lib import RQP_RUNNING
from .solver import Solver


@dataclass
class Request:
    rid: int
    family: int
    t_arrival: float  # seconds since the start of the run
    x0: np.ndarray
    t_done: float = float("nan")
    status: int = -1
    iterations: int = 0
    x: np.ndarray | None = None


@dataclass
class Family:
    """One QP family: its batched handle, slot bookkeeping and warm-start source."""

    solver: Solver
    stage: int                  # entries per horizon stage of x and of the constraint rows
    nx: int
    free: list = field(default_factory=list)
    busy: dict = field(default_factory=dict)  # slot -> Request
    queue: collections.deque = field(default_factory=collections.deque)
    pin: int | None = None      # slot holding the family's most recent solution
    single: Solver | None = None  # optional single-instance handle for light load

    @classmethod
    def from_mpc(cls, prob, slots: int, precision: str = "fp32", keep_x: bool = False, **settings):
        zq = np.zeros((slots, prob.n))
        lo = np.repeat(prob.lo[None, :], slots, axis=0)
        hi = np.repeat(prob.hi[None, :], slots, axis=0)
        s = Solver(prob.P, zq, prob.A, lo, hi, precision=precision, engine="batch", **settings)
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        fam = cls(solver=s, stage=prob.nu, nx=prob.nx)
        fam.free = list(range(slots))
        fam.keep_x = keep_x
        return fam

    def attach_single(self, prob, **settings):
        """Single-instance handle (FP32) of the same family, for light-load sequence launches."""
        q, l, u = prob.instance(np.zeros(prob.nx))
        s = Solver(prob.P, q, prob.A, l, u, precision="fp32", engine="single", **settings)
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        self.single = s
        return self


class Server:
    """Serves requests over families with continuous batching on one device stream."""

    def __init__(self, families: list[Family], n_checks: int = 1, warm: bool = True, light: int = 8):
        """light: a family with at most this many queued requests and no busy slot is served by
        a sequence launch of its single-instance handle (if attached)."""
        self.families = families
        self.n_checks = n_checks
        self.warm = warm
        self.light = light

    def _light_step(self, fam: Family):
        """Solve the family's whole (short) queue in one single-instance sequence launch."""
        reqs = list(fam.queue)
        fam.queue.clear()
        x0 = torch.tensor(np.stack([r.x0 for r in reqs]), dtype=torch.float64, device=fam.single.device)
        out = fam.single.solve_sequence(x0)
        return reqs, out

    def _admit(self, fam: Family):
        k = min(len(fam.queue), len(fam.free))
        if k == 0:
            return
        reqs = [fam.queue.popleft() for _ in range(k)]
        slots = [fam.free.pop() for _ in range(k)]
        x0 = torch.tensor(np.stack([r.x0 for r in reqs]), dtype=torch.float64, device=fam.solver.device)
        fam.solver.load_slots_x0(slots, x0)
        src = fam.pin if (self.warm and fam.pin is not None) else -1
        fam.solver.admit(slots, src_slot=src, shift_x=fam.stage, shift_y=fam.stage)
        for s, r in zip(slots, reqs):
            fam.busy[s] = r

    def _retire(self, fam: Family, now: float):
        if not fam.busy:
            return
        status = fam.solver.status.cpu().numpy()
        iters = fam.solver.iterations.cpu().numpy()
        done = [s for s in fam.busy if status[s] != RQP_RUNNING]
        if not done:
            return
        xs = fam.solver.x.cpu().numpy() if getattr(fam, "keep_x", False) else None
        for s in done:
            r = fam.busy.pop(s)
            r.t_done, r.status, r.iterations = now, int(status[s]), int(iters[s])
            if xs is not None:
                r.x = xs[s].astype(np.float64)
        # the newest solution becomes the warm-start source; the previous source slot is freed
        newest = max(done)
        if fam.pin is not None:
            fam.free.append(fam.pin)
        fam.pin = newest
        fam.free.extend(s for s in done if s != newest)

    def run(self, requests: list[Request], time_limit: float = 60.0) -> list[Request]:
        """Serve requests in arrival order (open loop); returns them with completion data."""
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or any(f.busy or f.queue for f in self.families):
            now = time.perf_counter() - t0
            if now > time_limit:
                break
            while pending and pending[0].t_arrival <= now:
                r = pending.popleft()
                self.families[r.family].queue.append(r)
            if not any(f.busy or f.queue for f in self.families):
                # idle until the next arrival
                time.sleep(max(0.0, pending[0].t_arrival - now) if pending else 0.0)
                continue
            light = []
            for fam in self.families:
                if fam.single is not None and not fam.busy and 0 < len(fam.queue) <= self.light:
                    light.append(self._light_step(fam))
                else:
                    self._admit(fam)
            for fam in self.families:
                if fam.busy:
                    fam.solver.step(self.n_checks)
            torch.cuda.synchronize()
            now = time.perf_counter() - t0
            for reqs, out in light:
                st = out["status"].cpu().numpy()
                it = out["iterations"].cpu().numpy()
                xs = out["x"].cpu().numpy()
                for i, r in enumerate(reqs):
                    r.t_done, r.status, r.iterations = now, int(st[i]), int(it[i])
                    r.x = xs[i].astype(np.float64)
            for fam in self.families:
                self._retire(fam, now)
        return requests


def serve_plain(solvers: list[Solver], requests: list[Request], time_limit: float = 60.0) -> list[Request]:
    """The same requests solved one at a time in arrival order on single-instance handles
    (one per family, parametric data set), cold starts."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = solvers[0].device
    for r in sorted(requests, key=lambda r: r.t_arrival):
        now = time.perf_counter() - t0
        if now > time_limit:
            break
        if r.t_arrival > now:
            time.sleep(r.t_arrival - now)
        s = solvers[r.family]
        s.update_x0_device(torch.tensor(r.x0[None, :], dtype=torch.float64, device=dev))
        s.solve()
        torch.cuda.synchronize()
        r.t_done = time.perf_counter() - t0
        r.status = int(s.status[0].item())
        r.iterations = int(s.iterations[0].item())
    return requests


def poisson_requests(rate: float, count: int, duration: float, families: list, seed: int) -> list[Request]:
    """Open-loop Poisson arrivals at `rate` per second, family chosen uniformly, fresh x0 per
    request from the family's x0 distribution (a callable family -> x0 given a Generator)."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        f = int(rng.integers(len(families)))
        out.append(Request(rid=i, family=f, t_arrival=t, x0=families[f](rng)))
    return out


def latency_summary(requests: list[Request], warmup: float = 0.0) -> dict:
    done = [r for r in requests if np.isfinite(r.t_done) and r.t_arrival >= warmup]
    if not done:
        return {"completed": 0}
    lat = np.array([r.t_done - r.t_arrival for r in done]) * 1e3
    span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
    return {
        "completed": len(done),
        "offered": sum(1 for r in requests if r.t_arrival >= warmup),
        "throughput_per_s": len(done) / span if span > 0 else float("nan"),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "solved_frac": float(np.mean([r.status == 1 for r in done])),
        "mean_iterations": float(np.mean([r.iterations for r in done])),
    }
