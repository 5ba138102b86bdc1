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

Admission by memory: with an HBM budget, a family's handles (layer weights for every penalty,
slot state, result buffers; ``footprint`` gives their bytes before any is created) are resident
only while they fit. A family with queued requests is loaded when its bytes fit beside the
resident ones, after unloading idle families (no busy slot) least recently used first; if it
cannot fit yet, families whose queued work is newer stop admitting, drain, and become idle.
Unloading spills a family to pinned host memory (``relu_qp_offload``) by default, so that
loading it again is a copy back (``relu_qp_restore``) rather than a new setup (factorisations);
its result tensors stay on the device and stay counted.

Latency is measured from a request's arrival time to the moment its result is on the host.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from ._lib import RQP_RUNNING
from .solver import Solver, footprint


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

    solver: Solver | None
    stage: int                  # entries per horizon stage of x and of the constraint rows
    nx: int
    free: list = field(default_factory=list)
    busy: dict = field(default_factory=dict)  # slot -> Request
    queue: collections.deque = field(default_factory=collections.deque)
    pin: int | None = None      # slot holding the family's most recent solution
    single: Solver | None = None  # optional single-instance handle for light load
    bytes: int = 0              # device bytes of the family's handles while resident
    residual: int = 0           # of which the result tensors (they stay when the family spills)
    last_used: float = 0.0
    keep_x: bool = False
    spec: dict = field(default_factory=dict)  # what load() builds
    spill: bool = True          # unload() offloads to pinned host memory instead of freeing
    spilled: bool = False

    @classmethod
    def from_mpc(cls, prob, slots: int, precision: str = "fp32", keep_x: bool = False, lazy: bool = False,
                 **settings):
        """lazy: only size the family (``footprint``); its handles are built by load()."""
        fam = cls(solver=None, stage=prob.nu, nx=prob.nx, keep_x=keep_x)
        fam.spec = dict(prob=prob, slots=slots, precision=precision, settings=settings, single=None)
        fp = footprint(prob.n, prob.m, prob.nx, batch=slots, precision=precision, engine="batch", **settings)
        fam.bytes, fam.residual = fp["resident"], fp["results"]
        if not lazy:
            fam.load()
        return fam

    @property
    def resident(self) -> bool:
        return self.solver is not None and not self.spilled

    def attach_single(self, prob, **settings):
        """Single-instance handle (FP32) of the same family, for light-load sequence launches."""
        self.spec["single"] = settings
        fp = footprint(prob.n, prob.m, prob.nx, batch=1, precision="fp32", engine="single", **settings)
        self.bytes += fp["resident"]
        self.residual += fp["results"]
        if self.resident:
            self._load_single()
        return self

    def _load_single(self):
        prob, settings = self.spec["prob"], self.spec["single"]
        # placeholder vectors (every request brings its own x0): q = 0, the limits' constant part
        s = Solver(prob.P, np.zeros(prob.n), prob.A, prob.lo, prob.hi, precision="fp32", engine="single", **settings)
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        self.single = s

    def load(self):
        """Build the family's device handles (setup on the device: factorizations per penalty)."""
        if self.resident:
            return
        if self.spilled:  # back from pinned host memory, exactly as it was
            for s in (self.solver, self.single):
                if s is not None:
                    s.restore()
            self.spilled = False
            self.free, self.busy, self.pin = list(range(self.spec["slots"])), {}, None
            return
        sp = self.spec
        prob, slots = sp["prob"], sp["slots"]
        zq = np.zeros((slots, prob.n))
        lo = np.repeat(prob.lo[None, :], slots, axis=0)
        hi = np.repeat(prob.hi[None, :], slots, axis=0)
        s = Solver(prob.P, zq, prob.A, lo, hi, precision=sp["precision"], engine="batch", **sp["settings"])
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        self.solver = s
        self.free, self.busy, self.pin = list(range(slots)), {}, None
        if sp["single"] is not None:
            self._load_single()

    def unload(self):
        """Take the family's handles out of HBM (no slot may be busy): spilled to pinned host
        memory, or freed; queued requests stay queued."""
        assert not self.busy, "unload with busy slots"
        self.pin, self.free = None, []
        if self.spill:
            for s in (self.solver, self.single):
                if s is not None:
                    s.offload()
            self.spilled = True
            return
        for s in (self.solver, self.single):
            if s is not None:
                s.close()
        self.solver, self.single = None, None
        torch.cuda.empty_cache()  # hand the result tensors' memory back for the next handle

    def close(self):
        for s in (self.solver, self.single):
            if s is not None:
                s.close()
        self.solver, self.single, self.spilled = None, None, False


def _staging(fam, name: str, rows: int, nx: int, device):
    """A family's pinned host buffer and device buffer of at least ``rows`` x0 rows (FP64),
    allocated once and kept with the family."""
    key = "_stage_" + name
    have = fam.__dict__.get(key)
    if have is None or have[0].shape[0] < rows:
        have = (torch.empty(rows, nx, dtype=torch.float64, pin_memory=True),
                torch.empty(rows, nx, dtype=torch.float64, device=device))
        fam.__dict__[key] = have
    return have


def _staging_results(fam, name: str, rows: int, solver):
    """Pinned host buffers for ``rows`` results (status, iterations, x) of a family."""
    key = "_res_" + name
    have = fam.__dict__.get(key)
    if have is None or have["status"].shape[0] < rows:
        have = dict(status=torch.empty(rows, dtype=torch.int32, pin_memory=True),
                    iterations=torch.empty(rows, dtype=torch.int32, pin_memory=True),
                    x=torch.empty(rows, solver.n, dtype=solver.dtype, pin_memory=True))
        fam.__dict__[key] = have
    return have


class MemoryPolicy:
    """Which families are resident under an HBM budget (host logic only).

    Works on any objects with ``bytes``, ``resident``, ``busy``, ``queue`` (requests with
    ``t_arrival``), ``last_used``, ``load()`` and ``unload()``."""

    def __init__(self, budget: int | None):
        self.budget = budget
        self.loads = 0
        self.evictions = 0
        self.peak = 0

    @staticmethod
    def _held(f) -> int:
        """Device bytes a family holds: all of them while resident, its result tensors while
        spilled, nothing while freed."""
        if f.resident:
            return f.bytes
        return getattr(f, "residual", 0) if getattr(f, "spilled", False) else 0

    @staticmethod
    def _freed(g) -> int:
        return g.bytes - (getattr(g, "residual", 0) if getattr(g, "spill", False) else 0)

    def used(self, families) -> int:
        return sum(self._held(f) for f in families)

    def check(self, families):
        if self.budget is None:
            return
        for f in families:
            # resident beside everything the other families keep while they are out of HBM
            others = sum(getattr(g, "residual", 0) for g in families if g is not f and getattr(g, "spill", False))
            if f.bytes + others > self.budget:
                raise ValueError(f"a family needs {f.bytes} bytes (+{others} kept by the others), more than the "
                                 f"budget {self.budget}")
        if self.used(families) > self.budget:
            raise ValueError("the families already resident exceed the budget")

    def _fit(self, fam, families) -> bool:
        used = self.used(families)
        if used + fam.bytes - self._held(fam) <= self.budget:
            return True
        head = fam.queue[0].t_arrival
        cands = [g for g in families if g is not fam and g.resident and not g.busy
                 and (not g.queue or g.queue[0].t_arrival > head)]
        cands.sort(key=lambda g: (bool(g.queue), g.last_used))
        need = fam.bytes - self._held(fam)  # a spilled family already holds its result tensors
        free_able = sum(self._freed(g) for g in cands)
        if used - free_able + need > self.budget:
            return False  # not even with every candidate gone: unload nothing yet
        for g in cands:
            g.unload()
            self.evictions += 1
            used -= self._freed(g)
            if used + need <= self.budget:
                break
        return True

    def schedule(self, families) -> set:
        """Load waiting families that fit (oldest queued request first); returns the ids of the
        resident families that must not admit new work this round (so that they drain)."""
        if self.budget is None:
            return set()
        gated = set()
        waiting = sorted((f for f in families if f.queue and not f.resident), key=lambda f: f.queue[0].t_arrival)
        for fam in waiting:
            if self._fit(fam, families):
                fam.load()
                self.loads += 1
                self.peak = max(self.peak, self.used(families))
                continue
            head = fam.queue[0].t_arrival
            for g in families:
                if g.resident and (not g.queue or g.queue[0].t_arrival > head):
                    gated.add(id(g))
            break
        return gated


class Server:
    """Serves requests over families with continuous batching on one device stream."""

    def __init__(self, families: list[Family], n_checks: int = 1, warm: bool = True, light: int = 8,
                 hbm_budget: int | None = None, spill: bool = True):
        """light: a family with at most this many queued requests and no busy slot is served by
        a sequence launch of its single-instance handle (if attached). hbm_budget: device bytes
        the families' handles may hold together (None: every family stays resident)."""
        self.families = families
        self.n_checks = n_checks
        self.warm = warm
        self.light = light
        self.memory = MemoryPolicy(hbm_budget)
        for f in families:
            f.spill = spill
        self.memory.check(families)
        if hbm_budget is None:
            for f in families:
                f.load()
        self.memory.peak = self.memory.used(families)

    def _light_step(self, fam: Family):
        """Solve the family's whole (short) queue in one single-instance sequence launch. The x0
        go through a pinned staging buffer, and the result tensors of each sequence length are
        allocated once per family (no fill kernels or allocations per request)."""
        reqs = list(fam.queue)
        fam.queue.clear()
        k = len(reqs)
        host, dev = _staging(fam, "light", self.light, fam.nx, fam.single.device)
        for i, r in enumerate(reqs):
            host[i].copy_(torch.from_numpy(r.x0))
        dev[:k].copy_(host[:k], non_blocking=True)
        outs = fam.__dict__.setdefault("_seq_out", {})
        if k not in outs:
            outs[k] = fam.single.sequence_slots(k)
        out = fam.single.solve_sequence(dev[:k], out=outs[k])
        # results come back through pinned buffers, read after the tick's synchronisation
        res = _staging_results(fam, "light", self.light, fam.single)
        res["status"][:k].copy_(out["status"], non_blocking=True)
        res["iterations"][:k].copy_(out["iterations"], non_blocking=True)
        res["x"][:k].copy_(out["x"], non_blocking=True)
        return reqs, res

    def _admit(self, fam: Family):
        k = min(len(fam.queue), len(fam.free))
        if k == 0:
            return
        reqs = [fam.queue.popleft() for _ in range(k)]
        slots = [fam.free.pop() for _ in range(k)]
        host, dev = _staging(fam, "admit", fam.spec["slots"], fam.nx, fam.solver.device)
        for i, r in enumerate(reqs):
            host[i].copy_(torch.from_numpy(r.x0))
        dev[:k].copy_(host[:k], non_blocking=True)
        fam.solver.load_slots_x0(slots, dev[:k])
        src = fam.pin if (self.warm and fam.pin is not None) else -1
        fam.solver.admit(slots, src_slot=src, shift_x=fam.stage, shift_y=fam.stage)
        for s, r in zip(slots, reqs):
            fam.busy[s] = r

    def _retire(self, fam: Family, now: float):
        if not fam.busy:
            return
        res = _staging_results(fam, "slots", fam.spec["slots"], fam.solver)
        status = res["status"].numpy()
        iters = res["iterations"].numpy()
        done = [s for s in fam.busy if status[s] != RQP_RUNNING]
        if not done:
            return
        xs = res["x"].numpy() if getattr(fam, "keep_x", False) else None
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
            gated = self.memory.schedule(self.families)
            light = []
            for fam in self.families:
                if not fam.resident or id(fam) in gated:
                    continue
                if fam.single is not None and not fam.busy and 0 < len(fam.queue) <= self.light:
                    light.append(self._light_step(fam))
                    fam.last_used = now
                else:
                    self._admit(fam)
            for fam in self.families:
                if fam.busy:
                    fam.solver.step(self.n_checks)
                    fam.last_used = now
            for fam in self.families:
                if fam.busy:  # slot states and counts to pinned buffers, read after the sync
                    res = _staging_results(fam, "slots", fam.spec["slots"], fam.solver)
                    res["status"].copy_(fam.solver.status, non_blocking=True)
                    res["iterations"].copy_(fam.solver.iterations, non_blocking=True)
                    if getattr(fam, "keep_x", False):
                        res["x"].copy_(fam.solver.x, non_blocking=True)
            torch.cuda.synchronize()
            now = time.perf_counter() - t0
            for reqs, res in light:
                st, it, xs = res["status"].numpy(), res["iterations"].numpy(), res["x"].numpy()
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
