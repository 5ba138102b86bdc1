"""Pins of the closed-loop MPC oracle (CPU only): the receding-horizon loop with exact solves
reproduces the Riccati feedback where no limit binds; the applied controls respect the limits
for any budget; the origin is an equilibrium; short budgets run no check and carry the penalty."""

import numpy as np

from oracle import admm
from oracle.closed_loop import closed_loop
from oracle.lqr import riccati_rollout
from workloads import make_config, x0_batch


def _settings(**kw):
    s = admm.Settings()
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_exact_solves_give_the_riccati_feedback():
    """Small states, no limit active: each step's QP is solved to 1e-11, and the applied control
    is the first control of the finite-horizon LQR problem from that state (Sec. II-C)."""
    prob = make_config("c0")
    x0 = 0.05 * x0_batch(prob.nx, 1, 31)[0]
    s = _settings(n_rho=8, eps_abs=1e-11, eps_rel=1e-11, max_iter=100000)
    xs, us, res = closed_loop(prob.P, prob.A, prob.F, prob.E, prob.lo, prob.hi, prob.A_dyn, prob.B, prob.nu,
                              x0, 12, s)
    assert all(r.status == admm.SOLVED for r in res)
    x = x0.copy()
    for k in range(12):
        u_r, _ = riccati_rollout(prob.A_dyn, prob.B, prob.Q, prob.R, prob.QN, prob.N, x)
        np.testing.assert_allclose(us[k], u_r[0], atol=1e-8)
        x = prob.A_dyn @ x + prob.B @ u_r[0]
        np.testing.assert_allclose(xs[k + 1], x, atol=1e-8)
    assert np.max(np.abs(us)) < 1.0  # the limits never bind here


def test_controls_respect_the_limits_for_any_budget():
    prob = make_config("c0")
    x0 = 8.0 * x0_batch(prob.nx, 1, 32)[0]
    for budget in (1, 2, 15, 25):
        s = _settings(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=budget)
        xs, us, res = closed_loop(prob.P, prob.A, prob.F, prob.E, prob.lo, prob.hi, prob.A_dyn, prob.B, prob.nu,
                                  x0, 40, s)
        assert np.all(np.abs(us) <= 1.0 + 1e-12), budget
        assert np.max(np.abs(us)) > 0.999  # large states: the limits bind
        assert all(r.status == admm.MAX_ITER and r.iterations == budget for r in res)


def test_origin_is_an_equilibrium():
    prob = make_config("c0")
    s = _settings(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=2)
    xs, us, _ = closed_loop(prob.P, prob.A, prob.F, prob.E, prob.lo, prob.hi, prob.A_dyn, prob.B, prob.nu,
                            np.zeros(prob.nx), 5, s)
    assert np.all(xs == 0.0) and np.all(us == 0.0)


def test_budgets_below_the_check_interval_run_no_check_and_carry_the_penalty():
    prob = make_config("c0")
    x0 = 8.0 * x0_batch(prob.nx, 1, 33)[0]
    s = _settings(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=2)
    _, _, res = closed_loop(prob.P, prob.A, prob.F, prob.E, prob.lo, prob.hi, prob.A_dyn, prob.B, prob.nu,
                            x0, 6, s)
    j0 = admm.rho_start_index(s)
    assert all(r.rho_hist == [] and r.rho_index == j0 for r in res)
    # a budget of 30 checks once (at 25) inside each step; the chosen index carries over
    s = _settings(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=30)
    _, _, res = closed_loop(prob.P, prob.A, prob.F, prob.E, prob.lo, prob.hi, prob.A_dyn, prob.B, prob.nu,
                            x0, 4, s)
    assert all(len(r.rho_hist) == 1 and r.rho_index == r.rho_hist[0] for r in res)
