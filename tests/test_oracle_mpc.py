"""Pins of the MPC input generator and of the oracle's per-solve update (CPU only).

The condensed QP of the paper's dense-MPC section must reproduce the exact unconstrained LQR
solution (Riccati recursion, Sec. II-C), for both the LQR-preconditioned and the plain
condensing (the reparametrisation u = -K x + du is exact, Sec. IV).
"""

import numpy as np
import pytest

import oracle
from oracle import admm
from oracle.lqr import dare_residual, riccati_rollout
from oracle.mpc_update import qp_vectors
from workloads import CONFIGS, make_config, random_mpc, x0_batch


@pytest.mark.parametrize("precondition", ["lqr", "none"])
def test_condensed_unconstrained_equals_riccati(precondition):
    prob = random_mpc(6, 2, 10, seed=0, precondition=precondition)
    x0 = x0_batch(6, 1, 3)[0]
    q, _, _ = prob.instance(x0)
    du = -np.linalg.solve(prob.P, q)
    us, xs = prob.trajectory(du, x0)
    us_r, xs_r = riccati_rollout(prob.A_dyn, prob.B, prob.Q, prob.R, prob.QN, prob.N, x0)
    np.testing.assert_allclose(us, us_r, atol=1e-9)
    np.testing.assert_allclose(xs, xs_r, atol=1e-9)


def test_lqr_gain_and_dynamics():
    prob = make_config("c0")
    assert dare_residual(prob.A_dyn, prob.B, prob.Q, prob.R, prob.K) < 1e-9
    assert np.max(np.abs(np.linalg.eigvals(prob.A_dyn))) == pytest.approx(1.05, rel=1e-12)
    assert np.max(np.abs(np.linalg.eigvals(prob.A_dyn - prob.B @ prob.K))) < 1.0
    # LQR preconditioning improves the condition number of the condensed Hessian
    plain = make_config("c0", precondition="none")
    assert np.linalg.cond(prob.P) < np.linalg.cond(plain.P)


def test_constraint_rows_are_the_limited_trajectory_entries():
    prob = make_config("c2", N=4)  # short horizon copy of the c2 recipe: u- and x-rows
    assert prob.m == 4 * 30 + 4 * 60
    x0 = x0_batch(60, 1, 5)[0]
    du = np.random.default_rng(0).standard_normal(prob.n)
    us, xs = prob.trajectory(du, x0)
    rows = prob.A @ du + prob.E @ x0
    np.testing.assert_allclose(rows[: 4 * 30], us.reshape(-1), atol=1e-10)
    np.testing.assert_allclose(rows[4 * 30 :], xs.reshape(-1), atol=1e-10)
    q, l, u = prob.instance(x0)
    np.testing.assert_allclose(l, -np.r_[np.ones(120), 2 * np.ones(240)] - prob.E @ x0)
    np.testing.assert_allclose(u - l, np.r_[2 * np.ones(120), 4 * np.ones(240)], atol=1e-12)


def test_reparametrisation_gives_same_constrained_solution():
    """Same constrained MPC optimum with and without the LQR reparametrisation."""
    lq = make_config("c0")
    pl = make_config("c0", precondition="none")
    x0 = 5.0 * x0_batch(6, 1, 11)[0]
    s = admm.Settings(eps_abs=1e-9, eps_rel=1e-9, n_rho=8, max_iter=40000)
    trajs = []
    for prob in (lq, pl):
        q, l, u = prob.instance(x0)
        r = oracle.solve(prob.P, q, prob.A, l, u, s)
        assert r.status == oracle.SOLVED
        trajs.append(prob.trajectory(r.x, x0))
    np.testing.assert_allclose(trajs[0][0], trajs[1][0], atol=1e-6)
    np.testing.assert_allclose(trajs[0][1], trajs[1][1], atol=1e-6)
    # the limits bind somewhere, so the clamp is exercised
    assert np.max(np.abs(trajs[0][0])) == pytest.approx(1.0, abs=1e-6)


def test_config_sizes():
    want = {"c0": (20, 20), "c1": (1600, 1600), "c2": (600, 1800)}
    for name, (n, m) in want.items():
        cfg = CONFIGS[name]
        nn = cfg["N"] * cfg["nu"]
        mm = nn + (cfg["N"] * cfg["nx"] if cfg.get("x_box") else 0)
        assert (nn, mm) == (n, m)


def test_oracle_update_matches_generator():
    prob = make_config("c0")
    x0s = x0_batch(6, 4, 9)
    qb, lb, ub = prob.instance(x0s)
    for i in range(4):
        q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, x0s[i])
        np.testing.assert_allclose(q, qb[i], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(l, lb[i], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(u, ub[i], rtol=1e-13, atol=1e-13)
