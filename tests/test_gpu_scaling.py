"""GPU parity of the Ruiz-scaled solve (settings.scaling > 0) against the oracle's scaled solve:
the kernel iterates on the scaled problem, judges termination on the original residuals and
writes the outputs in original units. Tolerances as for the unscaled path (1e-9 FP64, 1e-4
FP32 per vector, schedules replayed)."""

import numpy as np
import pytest

from oracle import admm
from oracle.mpc_update import qp_vectors
from oracle.scaling import ruiz, solve_scaled
from workloads import random_mpc, random_qp, x0_batch
from residual_check import assert_passes_fp64_test

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}


@pytest.fixture(scope="module")
def rq():
    import paper_2311_18056_amd as rq

    rq.lib()
    return rq


def _s(**kw):
    s = admm.Settings()
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _close(a, b, tol, what):
    err = np.max(np.abs(a - b))
    scale = max(np.max(np.abs(b)), 1.0)
    assert err <= tol * scale, f"{what}: |diff|={err:.3e} > {tol:.1e} * {scale:.3e}"


def _badly_scaled(seed, n=120, m_eq=20, m_ineq=40):
    P, q, A, l, u = random_qp(n, m_eq, m_ineq, seed=seed)
    S = np.diag(10.0 ** np.random.default_rng(seed).uniform(-1.5, 1.5, n))
    return S @ P @ S, S @ q, A @ S, l, u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(120, 20, 40), (30, 6, 20), (60, 10, 50)])
def test_scaled_per_iterate(rq, prec, shape):
    """n + m = 180 (persistent kernel), 56 and 120 (single-workgroup kernel, both lane shapes)."""
    P, q, A, l, u = _badly_scaled(31, *shape)
    sol = rq.Solver(P, q, A, l, u, precision=prec, n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=200, scaling=10)
    assert (sol.launch()[0] == 1) == (sum(shape) <= 128)
    sol.solve()
    r = sol.result()
    sol.close()
    ref = solve_scaled(P, q, A, l, u, _s(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=200), 10,
                       rho_replay=r["rho_hist"])
    for name in ("x", "z", "y"):
        _close(r[name], getattr(ref, name), TOL[prec], name)
    # the per-check primal residuals are the original problem's
    got, want = r["prim_res"][: len(ref.prim_res)], np.array(ref.prim_res)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert np.all(np.abs(got - want) <= tol * max(np.max(want), 1.0))


def test_scaled_updates_warm_start_and_parametric(rq):
    """q, l, u given later (host and device), a warm start in original units and the in-kernel
    update from x0 all pass through the scaling fixed at setup (D, E and c from the setup q)."""
    import torch

    prob = random_mpc(12, 4, 10, seed=5, precondition="none")
    x0 = 6.0 * x0_batch(prob.nx, 3, 77)
    q0, l0, u0 = prob.instance(x0[0])
    scaling = ruiz(prob.P, q0, prob.A, 10)
    kw = dict(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=80)
    sol = rq.Solver(prob.P, q0, prob.A, l0, u0, precision="fp64", scaling=10, **kw)
    sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    # host update
    q1, l1, u1 = prob.instance(x0[1])
    sol.update(q1, l1, u1)
    sol.solve()
    r = sol.result()
    ref = solve_scaled(prob.P, q1, prob.A, l1, u1, _s(**kw), 0, scaling=scaling, rho_replay=r["rho_hist"])
    for name in ("x", "z", "y"):
        _close(r[name], getattr(ref, name), 1e-9, "host update " + name)
    # warm start in original units from that solution, device update of q, l, u
    q2, l2, u2 = prob.instance(x0[2])
    sol.warm_start(ref.x, ref.y, ref.rho_index)
    dev = lambda v: torch.tensor(v, dtype=torch.float64, device="cuda")  # noqa: E731
    sol.update_device(dev(q2), dev(l2), dev(u2))
    sol.solve()
    r = sol.result()
    ref2 = solve_scaled(prob.P, q2, prob.A, l2, u2, _s(**kw), 0, scaling=scaling, rho_replay=r["rho_hist"],
                        warm=(ref.x, ref.y, ref.rho_index))
    for name in ("x", "z", "y"):
        _close(r[name], getattr(ref2, name), 1e-9, "warm + device update " + name)
    # in-kernel update from x0 (parametric data scaled at set_parametric)
    sol.set_warm(False)
    sol.solve_x0(dev(x0[1][None, :]))
    r = sol.result()
    q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, x0[1])
    ref3 = solve_scaled(prob.P, q, prob.A, l, u, _s(**kw), 0, scaling=scaling, rho_replay=r["rho_hist"])
    for name in ("x", "z", "y"):
        _close(r[name], getattr(ref3, name), 1e-9, "solve_x0 " + name)
    sol.close()


def test_scaling_on_an_ill_conditioned_mpc_fp32(rq):
    """Plain condensing (no LQR reparametrisation, condition number ~1e4): the scaled FP32
    solve reaches eps 1e-3 on the original residuals (re-evaluated in FP64 on the CPU)."""
    prob = random_mpc(30, 10, 40, seed=60, precondition="none")
    x0 = 20.0 * x0_batch(prob.nx, 1, 70)[0]
    q, l, u = prob.instance(x0)
    out = {}
    for sc in (0, 10):
        sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp32", n_rho=8, max_iter=4000, scaling=sc)
        sol.solve()
        out[sc] = sol.result()
        sol.close()
    r = out[10]
    assert r["status"] == rq.RQP_SOLVED
    x, z, y = (r[k].astype(np.float64) for k in ("x", "z", "y"))
    assert_passes_fp64_test(prob.P, q, prob.A, x, z, y, what="plain-condensed FP32, Ruiz scaling")
    xs = admm.solve(prob.P, q, prob.A, l, u, _s(n_rho=8, eps_abs=1e-10, eps_rel=1e-10, max_iter=400000)).x
    for sc in (0, 10):
        err = np.max(np.abs(out[sc]["x"] - xs)) / max(np.max(np.abs(xs)), 1.0)
        print(f"\nplain-condensed n={prob.n}, FP32, scaling {sc}: status {int(out[sc]['status'])}, "
              f"{int(out[sc]['iterations'])} iterations, solution error {err:.2e}")


# --------------------------------------------------------------------------- batched engine
# One scaling serves a whole batch: D and E come from P and A, which the instances share, and
# the cost scale c from the largest |q| entry over the setup instances (the oracle's ruiz with
# the stacked q gives the same (D, E, c)). The layer runs on the scaled problem; the check
# evaluates the original problem at the outputs (the unscaled iterates rounded to FP32).


def _dev(a):
    import torch

    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16x3", 5e-3)])
def test_batched_scaled_per_iterate(rq, prec, tol):
    """Badly scaled problem (n + m = 120), four instances with their own q, 100 iterations; each
    against the oracle's scaled solve with the batch's scaling and its schedule replayed."""
    P, q0, A, l0, u0 = _badly_scaled(33, 60, 0, 60)
    B = 4
    rng = np.random.default_rng(8)
    Q = q0[None, :] * (1.0 + 0.3 * rng.standard_normal((B, 60)))
    L, U = np.repeat(l0[None, :], B, 0), np.repeat(u0[None, :], B, 0)
    kw = dict(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=100)
    sol = rq.Solver(P, Q, A, L, U, precision=prec, engine="batch", scaling=10, **kw)
    sol.solve()
    r = sol.result()
    sol.close()
    scaling = ruiz(P, Q, A, 10)
    worst = 0.0
    for b in range(B):
        ref = solve_scaled(P, Q[b], A, L[b], U[b], _s(**kw), 0, scaling=scaling,
                           rho_replay=r["rho_hist"][b][:4].tolist())
        assert r["status"][b] == rq.RQP_MAX_ITER and r["iterations"][b] == 100
        for name in ("x", "z", "y"):
            worst = max(worst, np.max(np.abs(r[name][b] - getattr(ref, name))) / max(np.max(np.abs(getattr(ref, name))), 1.0))
            _close(r[name][b], getattr(ref, name), tol, f"{prec} instance {b} {name}")
        got, want = r["prim_res"][b][:4], np.array(ref.prim_res)
        assert np.all(np.abs(got - want) <= tol * max(np.max(want), 1.0)), (prec, b, got, want)
    print(f"\n{prec}: worst per-vector relative error, scaled batch vs oracle = {worst:.3e}")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batched_scaling_on_an_ill_conditioned_mpc(rq, prec):
    """Plain condensing (condition number ~1e4), six initial states: every instance stops SOLVED
    and its returned x, z, y pass the FP64 test of the original problem at 1.0 x eps."""
    prob = random_mpc(30, 10, 40, seed=60, precondition="none")
    B = 6
    x0 = 20.0 * x0_batch(prob.nx, B, 71)
    q, l, u = prob.instance(x0)
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision=prec, engine="batch", n_rho=8, max_iter=4000, scaling=10)
    sol.solve()
    r = sol.result()
    sol.close()
    for b in range(B):
        assert r["status"][b] == rq.RQP_SOLVED, (prec, b, int(r["status"][b]), int(r["iterations"][b]))
        x, z, y = (r[k][b].astype(np.float64) for k in ("x", "z", "y"))
        assert_passes_fp64_test(prob.P, q[b], prob.A, x, z, y, what=f"{prec} scaled batch instance {b}")


def test_batched_scaled_updates_warm_start_and_parametric(rq):
    """Host update of q, l, u, a warm start in original units and the in-kernel update from x0,
    all through the scaling fixed at setup."""
    prob = random_mpc(12, 4, 10, seed=5, precondition="none")
    B = 3
    x0 = 6.0 * x0_batch(prob.nx, 2 * B, 78)
    q0, l0, u0 = prob.instance(x0[:B])
    scaling = ruiz(prob.P, q0, prob.A, 10)
    kw = dict(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=75)
    sol = rq.Solver(prob.P, q0, prob.A, l0, u0, precision="fp32", engine="batch", scaling=10, **kw)
    sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    q1, l1, u1 = prob.instance(x0[B:])
    sol.update(q1, l1, u1)
    sol.solve()
    r = sol.result()
    refs = []
    for b in range(B):
        ref = solve_scaled(prob.P, q1[b], prob.A, l1[b], u1[b], _s(**kw), 0, scaling=scaling,
                           rho_replay=r["rho_hist"][b][:3].tolist())
        for name in ("x", "z", "y"):
            _close(r[name][b], getattr(ref, name), 1e-4, f"host update, instance {b} {name}")
        refs.append(ref)
    xw, yw = np.stack([f.x for f in refs]), np.stack([f.y for f in refs])
    sol.warm_start(xw, yw, 3)
    sol.update_x0_device(_dev(x0[:B]))
    sol.solve()
    r = sol.result()
    sol.close()
    for b in range(B):
        q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, x0[b])
        ref = solve_scaled(prob.P, q, prob.A, l, u, _s(**kw), 0, scaling=scaling, warm=(xw[b], yw[b], 3),
                           rho_replay=r["rho_hist"][b][:3].tolist())
        for name in ("x", "z", "y"):
            _close(r[name][b], getattr(ref, name), 1e-4, f"warm + x0 update, instance {b} {name}")


def test_batched_scaled_slots(rq):
    """Serving slots of a scaled handle: a slot loaded from x0 equals the same request solved alone
    (bit for bit, same scaling: q = 0 at setup in both); a slot loaded from device q, l, u rows and
    a warm admission shifted by one stage (entries change rows, hence units) match the oracle."""
    prob = random_mpc(12, 4, 10, seed=5, precondition="none")
    nu = prob.nu
    kw = dict(precision="fp32", n_rho=8, scaling=10)
    B = 4

    def handle(nb):
        s = rq.Solver(prob.P, np.zeros((nb, prob.n)), prob.A, np.repeat(prob.lo[None], nb, 0),
                      np.repeat(prob.hi[None], nb, 0), engine="batch", **kw)
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        return s

    def run(sol, slots):
        out = {}
        for _ in range(400):
            sol.step(1)
            r = sol.result()
            for s in slots:
                if s not in out and r["status"][s] != rq.RQP_RUNNING:
                    it = int(r["iterations"][s])
                    out[s] = dict(x=r["x"][s].copy(), y=r["y"][s].copy(), z=r["z"][s].copy(), iterations=it,
                                  status=int(r["status"][s]), rho_index=int(r["rho_index"][s]),
                                  rho_hist=r["rho_hist"][s][: -(-it // 25)].tolist())
            if len(out) == len(slots):
                return out
        raise AssertionError("slots did not finish")

    x0 = 6.0 * x0_batch(prob.nx, 3, 79)
    scaling = ruiz(prob.P, np.zeros(prob.n), prob.A, 10)
    sol = handle(B)
    q1, l1, u1 = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, x0[1])
    sol.load_slots_x0([1], _dev(x0[:1]))
    sol.load_slots([2], q=_dev(q1[None]), l=_dev(l1[None]), u=_dev(u1[None]))
    sol.admit([1, 2])
    d = run(sol, [1, 2])
    solo = handle(1)
    solo.update_x0_device(_dev(x0[:1]))
    solo.solve()
    r1 = solo.result(0)
    solo.close()
    assert d[1]["status"] == r1["status"] == rq.RQP_SOLVED and d[1]["iterations"] == r1["iterations"]
    for name in ("x", "y", "z"):
        assert np.array_equal(d[1][name], r1[name]), name
    s = _s(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=d[2]["iterations"])
    ref = solve_scaled(prob.P, q1, prob.A, l1, u1, s, 0, scaling=scaling, rho_replay=d[2]["rho_hist"])
    for name in ("x", "y", "z"):
        _close(d[2][name], getattr(ref, name), 1e-4, "slot from q, l, u rows " + name)
    # warm admission from slot 1, shifted by one stage
    src = d[1]
    sol.load_slots_x0([3], _dev(x0[2:3]))
    sol.admit([3], src_slot=1, shift_x=nu, shift_y=nu)
    d3 = run(sol, [3])[3]
    sol.close()
    xs = np.concatenate([src["x"][nu:], np.zeros(nu)])
    ys = np.concatenate([src["y"][nu:], np.zeros(nu)])
    q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, x0[2])
    s = _s(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=d3["iterations"])
    ref = solve_scaled(prob.P, q, prob.A, l, u, s, 0, scaling=scaling, warm=(xs, ys, src["rho_index"]),
                       rho_replay=d3["rho_hist"])
    for name in ("x", "y", "z"):
        _close(d3[name], getattr(ref, name), 1e-4, "shifted warm admission " + name)
