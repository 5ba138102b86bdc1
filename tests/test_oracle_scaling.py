"""Pins of the Ruiz equilibration in the oracle (CPU only): the equilibration property, the
exactness of the change of variables (brute force, closed form), unscaled termination, and the
identity scaling reproducing the unscaled solve."""

import numpy as np

from oracle import admm
from oracle.bruteforce import solve_qp_enumerate
from oracle.scaling import ruiz, scale_problem, solve_scaled
from workloads import random_box_qp, random_qp


def _s(**kw):
    s = admm.Settings()
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_equilibration_drives_kkt_columns_to_unit_norm():
    P, q, A, l, u = random_qp(30, 5, 20, seed=3)
    err = []
    for it in (1, 10, 60):
        D, E, c = ruiz(P, q, A, it, cost=False)
        assert c == 1.0 and np.all(D > 0) and np.all(E > 0)
        Pb, _, Ab, _, _ = scale_problem(P, q, A, l, u, D, E, 1.0)
        cols = np.r_[np.maximum(np.abs(Pb).max(0), np.abs(Ab).max(0)), np.abs(Ab).max(1)]
        err.append(np.max(np.abs(cols - 1.0)))
    assert err[0] > err[1] > err[2] and err[2] < 1e-12


def test_cost_scaling_normalises_the_cost():
    P, q, A, l, u = random_qp(20, 4, 6, seed=4)
    D, E, c = ruiz(P, 50.0 * q, A, 10)
    Pb, qb, _, _, _ = scale_problem(P, 50.0 * q, A, l, u, D, E, c)
    # after the last pass, max(mean column norm of P, ||q||_inf) is 1
    assert abs(max(np.mean(np.abs(Pb).max(0)), np.max(np.abs(qb))) - 1.0) < 1e-12


def test_scaled_solve_matches_brute_force():
    for seed in range(4):
        P, q, A, l, u = random_qp(6, 1, 5, seed=20 + seed)
        rng = np.random.default_rng(seed)
        S = np.diag(10.0 ** rng.uniform(-1.5, 1.5, 6))  # badly scaled variables
        P2, q2, A2 = S @ P @ S, S @ q, A @ S
        r = solve_scaled(P2, q2, A2, l, u, _s(n_rho=8, eps_abs=1e-11, eps_rel=1e-11, max_iter=400000), 10)
        assert r.status == admm.SOLVED
        x_bf = solve_qp_enumerate(P2, q2, A2, l, u)[0]
        np.testing.assert_allclose(r.x, x_bf, atol=1e-7 * max(1.0, np.max(np.abs(x_bf))))


def test_scaled_box_qp_closed_form():
    P, q, A, l, u = random_box_qp(12, seed=6)
    r = solve_scaled(P, q, A, l, u, _s(n_rho=8, eps_abs=1e-12, eps_rel=1e-12, max_iter=100000), 10)
    x_star = np.clip(-q / np.diag(P), l, u)
    np.testing.assert_allclose(r.x, x_star, atol=1e-9)
    np.testing.assert_allclose(r.z, x_star, atol=1e-9)


def test_termination_is_on_the_original_residuals():
    P, q, A, l, u = random_qp(40, 10, 20, seed=7)
    rng = np.random.default_rng(1)
    S = np.diag(10.0 ** rng.uniform(-1, 1, 40))
    P2, q2, A2 = S @ P @ S, S @ q, A @ S
    r = solve_scaled(P2, q2, A2, l, u, _s(n_rho=8, eps_abs=1e-6, eps_rel=1e-6, max_iter=20000), 10)
    assert r.status == admm.SOLVED
    nm = admm.residual_norms(P2, q2, A2, r.x, r.z, r.y)
    assert abs(nm["r_p"] - r.prim_res[-1]) <= 1e-12 * max(1.0, nm["Ax"])
    assert abs(nm["r_d"] - r.dual_res[-1]) <= 1e-12 * max(1.0, nm["Px"], nm["Aty"], nm["q"])
    assert nm["r_p"] <= 1e-6 + 1e-6 * max(nm["Ax"], nm["z"])
    assert nm["r_d"] <= 1e-6 + 1e-6 * max(nm["Px"], nm["Aty"], nm["q"])


def test_identity_scaling_is_the_plain_solve():
    P, q, A, l, u = random_qp(25, 5, 10, seed=8)
    s = _s(n_rho=8, max_iter=300)
    a = admm.solve(P, q, A, l, u, s)
    b = solve_scaled(P, q, A, l, u, s, 0, scaling=(np.ones(25), np.ones(15), 1.0))
    assert a.iterations == b.iterations and a.rho_hist == b.rho_hist
    for name in ("x", "y", "z"):
        assert np.array_equal(getattr(a, name), getattr(b, name))
