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
