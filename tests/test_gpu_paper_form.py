"""GPU runs of the paper's literal layer v <- clamp(W v + b) (eq. gpu_update) against the oracle's
literal form (``step_L`` with the printed W and b), from v = 0: x, z and the lagged dual after a
fixed number of layers, 1e-9 in FP64 and 1e-4 in FP32 (relative, per vector)."""

import numpy as np
import pytest

from oracle import admm
from workloads import make_config, random_qp, x0_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import paper_2311_18056_amd as rq

    rq.lib()
    return rq


def _close(a, b, tol, what):
    err = np.max(np.abs(a - b))
    scale = max(np.max(np.abs(b)), 1.0)
    assert err <= tol * scale, f"{what}: |diff|={err:.3e} > {tol:.1e} * {scale:.3e}"


def _oracle_layers(P, q, A, l, u, iters, rho0=0.1, sigma=1e-6, rho_eq_scale=1e3):
    s = admm.Settings()
    s.sigma, s.n_rho, s.rho0, s.rho_eq_scale = sigma, 1, rho0, rho_eq_scale
    rv = admm.rho_vector(rho0, l == u, s)
    D = admm.kkt_inverse(P, A, sigma, rv)
    W = admm.paper_W(D, P, A, rv, sigma)
    b = admm.paper_b(D, A, q)
    n, m = P.shape[0], A.shape[0]
    v = np.zeros(n + 2 * m)
    for _ in range(iters):
        v = admm.step_L(v, W, b, n, m, l, u)
    return v[:n], v[n:n + m], v[n + m:]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_paper_form_matches_the_literal_oracle(rq, prec, tol):
    prob = make_config("c0")
    q, l, u = prob.instance(5.0 * x0_batch(prob.nx, 1, 1000)[0])
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision=prec, alpha=1.0, n_rho=1, rho0=0.1)
    sol.solve_paper_form(60)
    r = sol.result()
    sol.close()
    x, z, lam = _oracle_layers(prob.P, q, prob.A, l, u, 60)
    _close(r["x"], x, tol, "x")
    _close(r["z"], z, tol, "z")
    _close(r["y"], lam, tol, "lagged dual")
    assert r["iterations"] == 60 and r["status"] == rq.RQP_MAX_ITER


def test_paper_form_equality_rows_and_many_rows(rq):
    """Equality rows (1000 x penalty), n + 2m = 300 over several rows per workgroup, FP64, and the
    weights reused by a second call on updated data."""
    P, q, A, l, u = random_qp(100, 20, 80, seed=12)
    sol = rq.Solver(P, q, A, l, u, precision="fp64", alpha=1.0, n_rho=1, rho0=0.1)
    sol.solve_paper_form(40)
    r = sol.result()
    x, z, lam = _oracle_layers(P, q, A, l, u, 40)
    _close(r["x"], x, 1e-9, "x")
    _close(r["z"], z, 1e-9, "z")
    _close(r["y"], lam, 1e-9, "lagged dual")
    q2 = q + 0.3
    sol.update(q=q2)
    sol.solve_paper_form(25)
    r = sol.result()
    sol.close()
    x, z, lam = _oracle_layers(P, q2, A, l, u, 25)
    _close(r["x"], x, 1e-9, "x after update")
    _close(r["z"], z, 1e-9, "z after update")


def test_paper_form_c2_shape_fp32(rq):
    """The n = 600, m = 1800 family (n + 2m = 4200 rows), FP32, against the oracle's literal form."""
    prob = make_config("c2")
    q, l, u = prob.instance(3.0 * x0_batch(prob.nx, 1, 1020)[0])
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp32", alpha=1.0, n_rho=1, rho0=0.1)
    sol.solve_paper_form(30)
    r = sol.result()
    sol.close()
    x, z, lam = _oracle_layers(prob.P, q, prob.A, l, u, 30)
    _close(r["x"], x, 1e-4, "x")
    _close(r["z"], z, 1e-4, "z")
    _close(r["y"], lam, 1e-4, "lagged dual")


def test_paper_form_rules(rq):
    prob = make_config("c0")
    q, l, u = prob.instance(x0_batch(prob.nx, 1, 1000)[0])
    for kw in (dict(alpha=1.6, n_rho=1), dict(alpha=1.0, n_rho=8)):
        sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp64", **kw)
        with pytest.raises(rq.ReluQPError):
            sol.solve_paper_form(5)
        sol.close()
