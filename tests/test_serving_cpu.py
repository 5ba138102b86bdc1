"""Host logic of serving by memory (no GPU): the footprint query of the C ABI and the policy that
keeps problem families resident under an HBM budget, driven with stand-in families."""

import collections
from dataclasses import dataclass, field

import pytest


def test_footprint_properties():
    import paper_2311_18056_amd as rq

    n, m, nx = 300, 500, 12

    def fp(**kw):
        return rq.footprint(n, m, **kw)

    single32 = fp(precision="fp32", engine="single")["library"]
    single64 = fp(precision="fp64", engine="single")["library"]
    # FP64 doubles the layer and check matrices (one per penalty, plus the check matrix)
    L, ldw = n + m, (n + m + 3) // 4 * 4
    assert 2 * L * ldw * 4 <= single64 - single32 < single32
    grid1 = fp(precision="fp32", engine="single", n_rho=1)["library"]
    grid2 = fp(precision="fp32", engine="single", n_rho=2)["library"]
    assert grid2 - grid1 == L * ldw * 4 + 8  # + one grid value (the midpoint list stays one long)
    # parametric data: F (n x nx), E (m x nx), lo, hi in FP64
    with_p = fp(precision="fp32", engine="single")["library"]
    assert rq.footprint(n, m, nx, precision="fp32", engine="single")["library"] - with_p == (n + m) * nx * 8 + 2 * m * 8
    # batched: per-slot state grows linearly between padding steps of 128 slots
    b1 = fp(precision="bf16x3", engine="batch", batch=129)["library"]
    b2 = fp(precision="bf16x3", engine="batch", batch=130)["library"]
    b3 = fp(precision="bf16x3", engine="batch", batch=131)["library"]
    assert b2 - b1 == b3 - b2 > 0
    # the result tensors: x, y, z, three counters and three per-check histories per slot
    r = fp(precision="fp32", engine="batch", batch=7, max_iter=100, check_interval=25)["results"]
    assert r == 7 * ((n + 2 * m) * 4 + 12 + 4 * 20)
    assert fp(precision="fp32", engine="single")["setup_extra"] >= (3 * n * n + 2 * m * n + m * m) * 8


def test_footprint_rejects_bad_input():
    import paper_2311_18056_amd as rq

    with pytest.raises(rq.ReluQPError):
        rq.footprint(0, 5)
    with pytest.raises(rq.ReluQPError):
        rq.footprint(5, 5, alpha=2.5)


@dataclass
class _Req:
    t_arrival: float


@dataclass
class _Fam:
    name: str
    bytes: int
    resident: bool = False
    busy: dict = field(default_factory=dict)
    queue: collections.deque = field(default_factory=collections.deque)
    last_used: float = 0.0
    log: list = None

    def load(self):
        assert not self.resident
        self.resident = True
        self.log.append(("load", self.name))

    def unload(self):
        assert self.resident and not self.busy
        self.resident = False
        self.log.append(("unload", self.name))


def _fams(sizes, log):
    return [_Fam(name=k, bytes=v, log=log) for k, v in sizes.items()]


def test_policy_loads_what_fits_and_evicts_idle_lru():
    from paper_2311_18056_amd.serving import MemoryPolicy

    log = []
    a, b, c = _fams({"a": 40, "b": 50, "c": 30}, log)
    pol = MemoryPolicy(100)
    fams = [a, b, c]
    a.queue.append(_Req(0.0))
    b.queue.append(_Req(0.1))
    assert pol.schedule(fams) == set()
    assert a.resident and b.resident and pol.used(fams) == 90
    # c needs 30: a and b are idle (their queues were taken), a is least recently used
    a.queue.clear()
    b.queue.clear()
    a.last_used, b.last_used = 1.0, 2.0
    c.queue.append(_Req(0.5))
    assert pol.schedule(fams) == set()
    assert c.resident and not a.resident and b.resident
    assert log[-2:] == [("unload", "a"), ("load", "c")]
    assert pol.evictions == 1 and pol.loads == 3 and pol.peak <= 100


def test_policy_never_evicts_busy_families_and_gates_newer_work():
    from paper_2311_18056_amd.serving import MemoryPolicy

    log = []
    a, b = _fams({"a": 60, "b": 60}, log)
    pol = MemoryPolicy(100)
    fams = [a, b]
    a.queue.append(_Req(0.0))
    pol.schedule(fams)
    a.queue.clear()
    a.busy = {0: "r"}
    # b waits behind busy a; a has newer queued work -> a is held back so it drains
    b.queue.append(_Req(1.0))
    a.queue.append(_Req(2.0))
    assert pol.schedule(fams) == {id(a)}
    assert a.resident and not b.resident
    # a's queued work older than b's head is not held back
    a.queue.appendleft(_Req(0.5))
    assert pol.schedule(fams) == set()
    a.queue.popleft()
    # a drains: b is loaded in a's place, a's newer request waits for its turn
    a.busy = {}
    assert pol.schedule(fams) == set()
    assert b.resident and not a.resident and pol.peak <= 100
    assert log == [("load", "a"), ("unload", "a"), ("load", "b")]


def test_policy_unloads_nothing_when_the_newcomer_cannot_fit_anyway():
    from paper_2311_18056_amd.serving import MemoryPolicy

    log = []
    a, b, c = _fams({"a": 50, "b": 40, "c": 70}, log)
    pol = MemoryPolicy(100)
    fams = [a, b, c]
    a.queue.append(_Req(0.0))
    b.queue.append(_Req(0.0))
    pol.schedule(fams)
    a.queue.clear()
    b.queue.clear()
    b.busy = {1: "r"}  # b (40) must stay; even without a, 40 + 70 > 100
    c.queue.append(_Req(1.0))
    assert pol.schedule(fams) == {id(a), id(b)}
    assert a.resident and b.resident and not c.resident
    assert pol.evictions == 0


def test_policy_rejects_a_family_larger_than_the_budget():
    from paper_2311_18056_amd.serving import MemoryPolicy

    with pytest.raises(ValueError):
        MemoryPolicy(10).check(_fams({"a": 11}, []))
    MemoryPolicy(None).check(_fams({"a": 11}, []))


def test_policy_counts_what_spilled_families_keep():
    from paper_2311_18056_amd.serving import MemoryPolicy

    log = []
    a, b = _fams({"a": 60, "b": 60}, log)
    for f in (a, b):
        f.spill, f.residual = True, 5
    # 60 + 5 must fit: 64 is too small
    with pytest.raises(ValueError):
        MemoryPolicy(64).check([a, b])
    pol = MemoryPolicy(70)
    pol.check([a, b])
    a.queue.append(_Req(0.0))
    pol.schedule([a, b])
    a.queue.clear()
    b.queue.append(_Req(1.0))
    a.spilled = False
    orig = a.unload

    def spill_a():
        orig()
        a.spilled = True

    a.unload = spill_a
    assert pol.schedule([a, b]) == set()
    assert b.resident and not a.resident and pol.used([a, b]) == 65 and pol.peak <= 70
