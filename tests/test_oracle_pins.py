"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a closed form, brute force,
the paper's printed weight matrix W, the paper's five-variable iteration, or OSQP's KKT-system
form. Together they catch a dropped term, a wrong sign or index, or a transposed operand in
any step of the iteration.
"""

import numpy as np
import pytest

import oracle
from oracle import admm
from oracle.bruteforce import solve_qp_enumerate
from workloads import random_box_qp, random_qp


def _rand_qp(rng, n, m, eq_rows=0):
    M = rng.standard_normal((n, n))
    P = M.T @ M / n + 0.1 * np.eye(n)
    q = rng.standard_normal(n)
    A = rng.standard_normal((m, n))
    xf = rng.standard_normal(n) * 0.3
    w = rng.uniform(0.05, 0.5, m)
    l, u = A @ xf - w, A @ xf + w
    l[:eq_rows] = u[:eq_rows] = (A @ xf)[:eq_rows]
    return P, q, A, l, u


# --------------------------------------------------------------------------- projection


def test_two_relu_clamp_identity():
    rng = np.random.default_rng(0)
    t = rng.standard_normal(1000) * 3
    l = rng.standard_normal(1000)
    u = l + np.abs(rng.standard_normal(1000))
    u[:100] = l[:100]  # l == u rows
    np.testing.assert_allclose(admm.clamp_two_relu(t, l, u), admm.clamp(t, l, u), rtol=0, atol=1e-15)
    # infinite bounds: the clamp is the identity / one-sided
    inf = np.full(1000, np.inf)
    np.testing.assert_array_equal(admm.clamp(t, -inf, inf), t)
    np.testing.assert_array_equal(admm.clamp(t, l, inf), np.maximum(t, l))
    # exact: the box is hit exactly, never overshot
    z = admm.clamp(t, l, u)
    assert np.all(z >= l) and np.all(z <= u)
    # NaN propagates through the projection
    assert np.isnan(admm.clamp(np.array([np.nan]), np.array([-1.0]), np.array([1.0]))[0])


# --------------------------------------------------------------------------- penalty grid


def test_rho_grid_closed_form():
    s = admm.Settings(n_rho=8, rho_min=1e-3, rho_max=1e3, rho0=0.1)
    g = admm.rho_grid(s)
    ratio = 10 ** (6 / 7)
    np.testing.assert_allclose(g, 1e-3 * ratio ** np.arange(8), rtol=1e-14)
    np.testing.assert_allclose(g[[1, 2, 3, 4, 5, 6]], [7.197e-3, 5.179e-2, 0.3728, 2.683, 19.31, 138.9], rtol=1e-3)
    assert admm.rho_start_index(s) == 2  # 0.1 -> 0.05179 (log distance 0.659 vs 1.31)
    assert admm.rho_grid(admm.Settings(n_rho=1, rho0=0.1))[0] == 0.1


def test_rho_nearest_and_ties():
    grid = np.array([1.0, 100.0])
    assert admm.nearest_rho_index(grid, 10.0) == 0  # exact tie in log distance -> smaller
    assert admm.nearest_rho_index(grid, 10.5) == 1
    assert admm.nearest_rho_index(grid, 1e-9) == 0 and admm.nearest_rho_index(grid, 1e9) == 1


def test_rho_hat_hand_norms():
    # eq. rho_update with hand-set norms: rho * sqrt(r_p * max(Px, Aty, q, 1e-4) / (r_d * max(Ax, z, 1e-4)))
    n = dict(r_p=4.0, r_d=1.0, Px=2.0, Aty=8.0, q=1.0, Ax=0.5, z=2.0)
    assert admm.rho_hat(0.1, n) == pytest.approx(0.1 * np.sqrt(4.0 * 8.0 / (1.0 * 2.0)), rel=1e-15)
    n0 = dict(r_p=1e-3, r_d=1e-3, Px=0.0, Aty=0.0, q=0.0, Ax=0.0, z=0.0)
    assert admm.rho_hat(2.0, n0) == pytest.approx(2.0, rel=1e-15)  # both floors at 1e-4


# --------------------------------------------------------------------------- the layer


def test_kkt_inverse():
    rng = np.random.default_rng(1)
    P, q, A, l, u = _rand_qp(rng, 12, 9, eq_rows=2)
    rv = admm.rho_vector(0.37, l == u, admm.Settings())
    D = admm.kkt_inverse(P, A, 1e-6, rv)
    K = P + 1e-6 * np.eye(12) + A.T @ np.diag(rv) @ A
    assert np.max(np.abs(D @ K - np.eye(12))) < 1e-10 * np.linalg.cond(K)
    assert np.array_equal(D, D.T)
    assert rv[0] == pytest.approx(370.0) and rv[5] == pytest.approx(0.37)
    with pytest.raises(np.linalg.LinAlgError):
        admm.kkt_inverse(-np.eye(3), np.zeros((1, 3)), 1e-6, np.ones(1))


def test_paper_W_equals_modified_admm_steps():
    """eq. gpu_update's W, b reproduce eqs. basic_lambda_update, basic_y_update and clamp."""
    rng = np.random.default_rng(2)
    n, m = 7, 5
    P, q, A, l, u = _rand_qp(rng, n, m)
    rv = rng.uniform(0.1, 3.0, m)  # any diagonal rho
    sigma = 1e-3
    D = np.linalg.inv(P + sigma * np.eye(n) + A.T @ np.diag(rv) @ A)
    W = admm.paper_W(D, P, A, rv, sigma)
    b = admm.paper_b(D, A, q)
    x, z, y = rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(m)
    # the three modified steps, composed directly
    lam_n = y + rv * (A @ x - z)
    x_n = np.linalg.solve(P + sigma * np.eye(n) + A.T @ np.diag(rv) @ A, -q + sigma * x + A.T @ (rv * z - lam_n))
    z_n = np.clip(A @ x_n + lam_n / rv, l, u)
    v = admm.step_L(np.concatenate([x, z, y]), W, b, n, m, l, u)
    np.testing.assert_allclose(v, np.concatenate([x_n, z_n, lam_n]), rtol=1e-11, atol=1e-11)


def _run_T(P, q, A, l, u, rv, sigma, alpha, k):
    lu = admm.full_kkt_lu(P, A, sigma, rv)
    n, m = P.shape[0], A.shape[0]
    x, z, y = np.zeros(n), np.zeros(m), np.zeros(m)
    out = []
    for _ in range(k):
        x, z, y = admm.step_T(x, z, y, lu, rv, q, A, l, u, sigma, alpha)
        out.append((x, z, y))
    return out


@pytest.mark.parametrize("alpha", [1.0, 1.6, 0.7])
def test_layer_form_R_equals_osqp_form_T(alpha):
    rng = np.random.default_rng(3)
    P, q, A, l, u = _rand_qp(rng, 10, 14, eq_rows=3)
    rv = admm.rho_vector(0.2, l == u, admm.Settings())
    sigma = 1e-6
    ref = _run_T(P, q, A, l, u, rv, sigma, alpha, 80)
    D = admm.kkt_inverse(P, A, sigma, rv)
    x, z, y = np.zeros(10), np.zeros(14), np.zeros(14)
    for k in range(80):
        x, z, y = admm.step_R(x, z, y, D, rv, q, A, l, u, sigma, alpha)
        for a, b_ in zip((x, z, y), ref[k]):
            assert np.max(np.abs(a - b_)) <= 1e-9 * max(np.max(np.abs(b_)), 1.0)


def test_paper_layer_L_equals_textbook_at_alpha_1():
    """The paper's layer carries the dual one step behind; with lam_0 shifted it is textbook ADMM."""
    rng = np.random.default_rng(4)
    n, m = 9, 11
    P, q, A, l, u = _rand_qp(rng, n, m)
    rv = np.full(m, 0.3)
    sigma = 1e-6
    ref = _run_T(P, q, A, l, u, rv, sigma, 1.0, 60)
    D = admm.kkt_inverse(P, A, sigma, rv)
    W = admm.paper_W(D, P, A, rv, sigma)
    b = admm.paper_b(D, A, q)
    x0, z0, y0 = np.zeros(n), np.zeros(m), np.zeros(m)
    v = np.concatenate([x0, z0, y0 - rv * (A @ x0 - z0)])
    for k in range(60):
        v = admm.step_L(v, W, b, n, m, l, u)
        x, z, lam_lag = v[:n], v[n : n + m], v[n + m :]
        xr, zr, yr = ref[k]
        assert np.max(np.abs(x - xr)) <= 1e-9 * max(np.max(np.abs(xr)), 1)
        assert np.max(np.abs(z - zr)) <= 1e-9 * max(np.max(np.abs(zr)), 1)
        # textbook dual = lagged dual + rho (A x - z)
        y = lam_lag + rv * (A @ x - z)
        assert np.max(np.abs(y - yr)) <= 1e-9 * max(np.max(np.abs(yr)), 1)


def test_mu_vanishes_after_one_iteration():
    """Sec. II-B remark: eqs. x_update and mu_update_gen force mu = 0 from the second iteration."""
    rng = np.random.default_rng(5)
    n, m = 8, 6
    H, g, G, c, d = _rand_qp(rng, n, m)
    rv = np.full(m, 0.5)
    sigma = 1e-2
    D = admm.kkt_inverse(H, G, sigma, rv)
    ybar, y, z = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(m)
    mu, lam = rng.standard_normal(n), rng.standard_normal(m)
    ybar, y, z, mu, lam = admm.step_paper5(ybar, y, z, mu, lam, D, rv, H, g, G, c, d, sigma)
    assert np.max(np.abs(mu)) < 1e-12
    # from here on the five-variable iteration is the three-variable one (alpha = 1)
    xr, zr, yr = y.copy(), z.copy(), lam.copy()
    for _ in range(30):
        ybar, y, z, mu, lam = admm.step_paper5(ybar, y, z, mu, lam, D, rv, H, g, G, c, d, sigma)
        xr, zr, yr = admm.step_R(xr, zr, yr, D, rv, g, G, c, d, sigma, 1.0)
        assert np.max(np.abs(mu)) < 1e-12
        np.testing.assert_allclose(y, xr, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(ybar, y, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(z, zr, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(lam, yr, rtol=1e-9, atol=1e-9)


# --------------------------------------------------------------------------- fixed points


def test_bruteforce_matches_box_closed_form():
    for seed in range(5):
        P, q, A, l, u = random_box_qp(6, seed)
        x, y = solve_qp_enumerate(P, q, A, l, u)
        d = np.diag(P)
        xs = np.clip(-q / d, l, u)
        np.testing.assert_allclose(x, xs, atol=1e-12)
        np.testing.assert_allclose(y, -(d * xs + q), atol=1e-12)


def test_oracle_box_qp_closed_form():
    s = admm.Settings(eps_abs=1e-11, eps_rel=1e-11, max_iter=20000, n_rho=8)
    for seed in range(3):
        P, q, A, l, u = random_box_qp(8, 100 + seed)
        r = oracle.solve(P, q, A, l, u, s)
        assert r.status == oracle.SOLVED
        xs = np.clip(-q / np.diag(P), l, u)
        np.testing.assert_allclose(r.x, xs, atol=1e-8)


@pytest.mark.parametrize("alpha", [1.0, 1.6])
@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_bruteforce(alpha, seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 8))
    m = int(rng.integers(1, 8))
    P, q, A, l, u = _rand_qp(rng, n, m, eq_rows=int(seed % 2))
    xs, ys = solve_qp_enumerate(P, q, A, l, u)
    s = admm.Settings(alpha=alpha, eps_abs=1e-10, eps_rel=1e-10, max_iter=50000, n_rho=8)
    r = oracle.solve(P, q, A, l, u, s)
    assert r.status == oracle.SOLVED
    np.testing.assert_allclose(r.x, xs, atol=1e-6 * max(1, np.max(np.abs(xs))))
    np.testing.assert_allclose(r.y, ys, atol=1e-5 * max(1, np.max(np.abs(ys))))


def test_unconstrained_closed_form():
    rng = np.random.default_rng(7)
    P, q, A, l, u = _rand_qp(rng, 10, 6)
    l[:] = -np.inf
    u[:] = np.inf
    r = oracle.solve(P, q, A, l, u, admm.Settings(eps_abs=1e-10, eps_rel=1e-10, max_iter=20000))
    assert r.status == oracle.SOLVED
    np.testing.assert_allclose(r.x, -np.linalg.solve(P, q), atol=1e-8)
    assert np.max(np.abs(r.y)) < 1e-8


def test_equality_constrained_closed_form():
    rng = np.random.default_rng(8)
    n, m = 10, 4
    P, q, A, l, u = _rand_qp(rng, n, m, eq_rows=m)
    K = np.block([[P, A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-q, l]))
    r = oracle.solve(P, q, A, l, u, admm.Settings(eps_abs=1e-10, eps_rel=1e-10, max_iter=20000, n_rho=8))
    assert r.status == oracle.SOLVED
    np.testing.assert_allclose(r.x, sol[:n], atol=1e-7)
    np.testing.assert_allclose(r.y, sol[n:], atol=1e-6)


def test_kkt_conditions_at_convergence():
    P, q, A, l, u = random_qp(40, 10, 10, seed=3)
    s = admm.Settings(eps_abs=1e-6, eps_rel=1e-6, n_rho=8, max_iter=20000)
    r = oracle.solve(P, q, A, l, u, s)
    assert r.status == oracle.SOLVED and r.iterations % 25 == 0
    nm = admm.residual_norms(P, q, A, r.x, r.z, r.y)
    assert nm["r_p"] <= 1e-6 + 1e-6 * max(nm["Ax"], nm["z"])
    assert nm["r_d"] <= 1e-6 + 1e-6 * max(nm["Px"], nm["Aty"], nm["q"])
    assert np.all(r.z >= l) and np.all(r.z <= u)
    # complementarity: y_i > 0 only at the upper bound, y_i < 0 only at the lower bound
    ineq = l < u
    up = r.y > 1e-6
    lo = r.y < -1e-6
    assert np.all(np.abs(r.z - u)[up & ineq] < 1e-9)
    assert np.all(np.abs(r.z - l)[lo & ineq] < 1e-9)


# --------------------------------------------------------------------------- solve-loop logic


def test_nonfinite_status():
    P, q, A, l, u = random_box_qp(5, 0)
    q = q.copy()
    q[2] = np.nan
    r = oracle.solve(P, q, A, l, u, admm.Settings())
    assert r.status == oracle.NONFINITE and r.iterations == 25


def test_fixed_iteration_mode_and_max_iter():
    P, q, A, l, u = random_qp(12, 3, 3, seed=1)
    r = oracle.solve(P, q, A, l, u, admm.Settings(eps_abs=0.0, eps_rel=0.0, max_iter=130))
    assert r.status == oracle.MAX_ITER and r.iterations == 130
    assert len(r.rho_hist) == 6  # checks at 25, 50, 75, 100, 125 and at max_iter = 130


def test_replay_own_schedule_is_identical():
    P, q, A, l, u = random_qp(30, 8, 8, seed=0)
    s = admm.Settings(n_rho=8, eps_abs=1e-7, eps_rel=1e-7, max_iter=3000)
    r1 = oracle.solve(P, q, A, l, u, s)
    assert len(set(r1.rho_hist)) > 1  # the schedule does move
    r2 = oracle.solve(P, q, A, l, u, s, rho_replay=r1.rho_hist)
    assert r2.iterations == r1.iterations and np.array_equal(r2.x, r1.x)


def test_warm_start_from_solution_stops_at_first_check():
    P, q, A, l, u = random_qp(20, 5, 5, seed=4)
    s = admm.Settings(n_rho=8, eps_abs=1e-5, eps_rel=1e-5, max_iter=5000)
    r1 = oracle.solve(P, q, A, l, u, s)
    assert r1.status == oracle.SOLVED
    r2 = oracle.solve(P, q, A, l, u, s, warm=(r1.x, r1.y, r1.rho_index))
    assert r2.status == oracle.SOLVED and r2.iterations == 25


def test_validation_errors():
    P, q, A, l, u = random_box_qp(3, 0)
    with pytest.raises(ValueError):
        oracle.solve(P, q, A, u, l - 10, admm.Settings())  # l > u
    with pytest.raises(ValueError):
        oracle.solve(P, q, A, l, u, admm.Settings(alpha=2.0))
    Pn = P.copy()
    Pn[0, 0] = np.inf
    with pytest.raises(ValueError):
        oracle.solve(Pn, q, A, l, u, admm.Settings())


# --------------------------------------------------------------------------- tolerance split
# The convergence criteria (Sec. III-C, eqs. primal and dual) compare each residual with its
# own tolerance; the relative part follows OSQP: the primal one scales with max(|Ax|, |z|),
# the dual one with max(|Px|, |A'y|, |q|). Two exact changes of units pin that split without
# restating it: scaling the cost by c (P, q, sigma, rho by c) keeps x and z and multiplies y
# by c; scaling the constraint rows by d (A, l, u by d, rho by 1/d^2) keeps x and multiplies
# z by d and y by 1/d. With eps_abs = 0 a correct split takes the same decision at every check
# under both; a split that puts any dual term into the primal tolerance (or the converse), or
# leaves out the relative part of either, stops at another iteration once c or d is 2^16.


def _scaled_solve(P, q, A, l, u, s, c=1.0, d=1.0):
    from dataclasses import replace

    s2 = replace(s, rho0=s.rho0 * c / (d * d), sigma=s.sigma * c)
    return oracle.solve(c * P, c * q, d * A, d * l, d * u, s2)


@pytest.mark.parametrize("c,d", [(2.0**16, 1.0), (2.0**-16, 1.0), (1.0, 2.0**16), (1.0, 2.0**-16)])
def test_tolerance_split_is_unit_invariant(c, d):
    P, q, A, l, u = random_qp(30, 8, 8, seed=5)
    s = admm.Settings(eps_abs=0.0, eps_rel=1e-5, n_rho=1, rho0=0.1, max_iter=4000)
    r0 = _scaled_solve(P, q, A, l, u, s)
    assert r0.status == oracle.SOLVED and r0.iterations >= 100  # several checks decide
    r1 = _scaled_solve(P, q, A, l, u, s, c, d)
    assert r1.status == oracle.SOLVED and r1.iterations == r0.iterations
    np.testing.assert_allclose(r1.x, r0.x, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r1.z / d, r0.z, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r1.y * d / c, r0.y, rtol=1e-9, atol=1e-12)


def test_tolerance_split_mistakes_are_caught(monkeypatch):
    """The pin above fails for a swapped split (a mistake planted in the oracle, on the CPU)."""
    P, q, A, l, u = random_qp(30, 8, 8, seed=5)
    s = admm.Settings(eps_abs=0.0, eps_rel=1e-5, n_rho=1, rho0=0.1, max_iter=4000)
    true_norms = admm.residual_norms

    def swapped(*args):
        nm = dict(true_norms(*args))
        nm["Ax"], nm["z"], nm["Px"], nm["Aty"], nm["q"] = nm["Px"], nm["Aty"], nm["Ax"], nm["z"], 0.0
        return nm

    monkeypatch.setattr(admm, "residual_norms", swapped)
    r0 = _scaled_solve(P, q, A, l, u, s)
    r1 = _scaled_solve(P, q, A, l, u, s, 2.0**16, 1.0)
    r2 = _scaled_solve(P, q, A, l, u, s, 1.0, 2.0**16)
    assert r1.iterations != r0.iterations or r2.iterations != r0.iterations
