"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same inputs.

Tolerances (per vector v in x, z, y): ||v_gpu - v_oracle||_inf <= tol * max(||v_oracle||_inf, 1),
tol = 1e-9 for FP64 and 1e-4 for FP32, over fixed iteration counts, with the penalty schedule
the GPU chose replayed in the oracle.
"""

import numpy as np
import pytest

import oracle
from oracle import admm
from oracle.mpc_update import qp_vectors
from residual_check import assert_passes_fp64_test
from workloads import make_config, random_qp, x0_batch

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}


@pytest.fixture(scope="module")
def rq():
    import paper_2311_18056_amd as rq

    rq.lib()
    return rq


@pytest.fixture(scope="module")
def c0():
    prob = make_config("c0")
    x0 = x0_batch(prob.nx, 4, 1000)
    return prob, x0


def _oracle_settings(**kw):
    s = admm.Settings()
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _close(a, b, tol, what=""):
    err = np.max(np.abs(a - b)) if a.size else 0.0
    scale = max(np.max(np.abs(b)) if b.size else 0.0, 1.0)
    assert err <= tol * scale, f"{what}: |diff|={err:.3e} > {tol:.1e} * {scale:.3e}"


def _compare(res, ref, tol):
    _close(res["x"], ref.x, tol, "x")
    _close(res["z"], ref.z, tol, "z")
    _close(res["y"], ref.y, tol, "y")


def _fixed_run(rq, P, q, A, l, u, prec, iters, grid=None, **kw):
    s = dict(eps_abs=0.0, eps_rel=0.0, max_iter=iters, precision=prec, **kw)
    sol = rq.Solver(P, q, A, l, u, **s)
    if grid is not None:
        sol.set_launch(grid)
    sol.solve()
    res = sol.result()
    sol.close()
    return res


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("iters", [1, 2, 3, 24, 25, 26, 57, 200])
def test_c0_fixed_rho_per_iterate(rq, c0, prec, iters):
    prob, x0 = c0
    q, l, u = prob.instance(5.0 * x0[0])  # scaled so that limits bind
    res = _fixed_run(rq, prob.P, q, prob.A, l, u, prec, iters)
    ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=iters))
    assert res["status"] == rq.RQP_MAX_ITER and res["iterations"] == iters
    _compare(res, ref, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c0_adaptive_rho_replayed(rq, c0, prec):
    prob, x0 = c0
    q, l, u = prob.instance(5.0 * x0[1])
    res = _fixed_run(rq, prob.P, q, prob.A, l, u, prec, 300, n_rho=8)
    assert len(res["rho_hist"]) == 12
    ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=300, n_rho=8),
                       rho_replay=res["rho_hist"])
    assert res["rho_index"] == ref.rho_index
    _compare(res, ref, TOL[prec])
    if prec == "fp64":
        # The FP64 path takes the oracle's own decisions for as long as the residuals are
        # resolvable; once both sit at rounding level (about 1e-15 here) the ratio in the
        # penalty rule is rounding noise and either choice is valid.
        own = oracle.solve(prob.P, q, prob.A, l, u,
                           _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=300, n_rho=8), record=True)
        resolvable = [c for c in range(len(own.rho_hist)) if min(own.prim_res[c], own.dual_res[c]) > 1e-10]
        assert len(resolvable) >= 4
        last = resolvable[-1]
        assert own.rho_hist[: last + 1] == res["rho_hist"][: last + 1]
        # the residuals are FP64 evaluations of iterates that agree to the per-iterate tolerance
        # (1e-9 relative), so they agree to 1e-7 relative plus 1e-9 times the row sums of |P|,
        # |A| and |A'| scaled by max(||v||, 1) at that check
        aP, aA = np.abs(prob.P), np.abs(prob.A)
        for c in range(len(own.prim_res)):
            if own.rho_hist[:c] != res["rho_hist"][:c]:
                break  # past the resolvable checks the two may take other (equally valid) penalties
            x, z, y = own.history[25 * (c + 1) - 1]
            sx, sy = max(np.max(np.abs(x)), 1.0), max(np.max(np.abs(y)), 1.0)
            bp = 1e-9 * (np.max(aA.sum(axis=1)) * sx + max(np.max(np.abs(z)), 1.0))
            bd = 1e-9 * np.max(aP.sum(axis=1) * sx + aA.sum(axis=0) * sy)
            assert abs(res["prim_res"][c] - own.prim_res[c]) <= 1e-7 * own.prim_res[c] + bp, c
            assert abs(res["dual_res"][c] - own.dual_res[c]) <= 1e-7 * own.dual_res[c] + bd, c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("grid", [3, 5, 17, 64, 180])
def test_launch_shapes_and_streamed_rows(rq, prec, grid):
    """Same result for any number of workgroups; few workgroups put many rows (register and
    streamed) on each, so every path of the row loop runs."""
    P, q, A, l, u = random_qp(120, 20, 40, seed=11)  # L = 180 rows, equality rows included
    res = _fixed_run(rq, P, q, A, l, u, prec, 60, grid=grid, n_rho=8)
    ref = oracle.solve(P, q, A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=60, n_rho=8),
                       rho_replay=res["rho_hist"])
    _compare(res, ref, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("grid", [1, 2, 7, 40])
def test_c0_launch_shapes(rq, c0, prec, grid):
    """The n = m = 20 instance on the persistent kernel (an explicit grid selects it), from one
    workgroup (every row its own, no exchange partner) up to one row per workgroup, per iterate
    against the oracle with limits binding."""
    prob, x0 = c0
    q, l, u = prob.instance(5.0 * x0[2])
    res = _fixed_run(rq, prob.P, q, prob.A, l, u, prec, 200, grid=grid)
    ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=200))
    assert res["status"] == rq.RQP_MAX_ITER and res["iterations"] == 200
    _compare(res, ref, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(1, 0, 1), (7, 2, 5), (20, 4, 16), (60, 8, 60), (61, 8, 60)])
def test_single_workgroup_sizes(rq, prec, shape):
    """Problems with n + m <= 128 run on one workgroup by default (lanes per row 64 down to 8,
    128 rows at the top, equality rows with their scaled penalty); one row more takes the
    persistent kernel. Per iterate against the oracle with the penalty schedule replayed."""
    n, m_eq, m_ineq = shape
    P, q, A, l, u = random_qp(n, m_eq, m_ineq, seed=100 + n)
    sol = rq.Solver(P, q, A, l, u, precision=prec, n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=150)
    L = n + m_eq + m_ineq
    assert sol.launch()[0] == (1 if L <= 128 else -(-L * 2 // 25))  # ceil(L / 12.5) above 128
    sol.solve()
    res = sol.result()
    sol.close()
    ref = oracle.solve(P, q, A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=150, n_rho=8),
                       rho_replay=res["rho_hist"])
    assert res["iterations"] == 150 and res["status"] == rq.RQP_MAX_ITER
    _compare(res, ref, TOL[prec])


def test_single_workgroup_matches_persistent(rq, c0):
    """The same c0 solve to eps 1e-3 in FP64 on the single-workgroup kernel and on the persistent
    one: equal iteration counts and penalty histories, iterates within the FP64 tolerance."""
    prob, x0 = c0
    q, l, u = prob.instance(5.0 * x0[3])
    out = []
    for grid in (0, 8):
        sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp64", n_rho=8)
        sol.set_launch(grid)
        assert sol.launch()[0] == (1 if grid == 0 else grid)
        sol.solve()
        out.append(sol.result())
        sol.close()
    a, b = out
    assert a["status"] == b["status"] == rq.RQP_SOLVED
    assert a["iterations"] == b["iterations"] and a["rho_hist"] == b["rho_hist"]
    for name in ("x", "y", "z"):
        _close(a[name], b[name], TOL["fp64"], name)


def test_abort_single_workgroup(rq):
    import time

    P, q, A, l, u = random_qp(20, 4, 16, seed=6)
    sol = rq.Solver(P, q, A, l, u, precision="fp64", eps_abs=0.0, eps_rel=0.0, max_iter=20_000_000)
    assert sol.launch()[0] == 1
    sol.solve()
    time.sleep(0.05)
    sol.abort()
    res = sol.result()
    sol.close()
    assert res["status"] == rq.RQP_ABORTED
    assert 0 < res["iterations"] < 20_000_000 and res["iterations"] % 25 == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c0_solves_to_tolerance(rq, c0, prec):
    prob, x0 = c0
    for i in range(3):
        q, l, u = prob.instance(5.0 * x0[i])
        sol = rq.Solver(prob.P, q, prob.A, l, u, precision=prec, n_rho=8)
        sol.solve()
        res = sol.result()
        sol.close()
        assert res["status"] == rq.RQP_SOLVED
        assert res["iterations"] % 25 == 0
        assert_passes_fp64_test(prob.P, q, prob.A, res["x"], res["z"], res["y"], what=f"c0 {prec} solve {i}")
        xs = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=1e-10, eps_rel=1e-10, n_rho=8,
                                                                    max_iter=40000)).x
        err = np.max(np.abs(res["x"] - xs)) / max(np.max(np.abs(xs)), 1.0)
        assert err < 5e-2, f"solution error {err:.2e}"


def test_c1_full_size_fp32_replayed(rq):
    """Config 1 shape (n = m = 1600, 8 penalties) in the launch configuration the benchmark
    times, 150 fixed iterations with the GPU's schedule replayed."""
    prob = make_config("c1")
    x0 = x0_batch(prob.nx, 1, 1001, scale=20.0)[0]
    q, l, u = prob.instance(x0)
    res = _fixed_run(rq, prob.P, q, prob.A, l, u, "fp32", 150, n_rho=8)
    ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=150, n_rho=8),
                       rho_replay=res["rho_hist"])
    _compare(res, ref, TOL["fp32"])


def test_c1_solution_quality_fp32(rq):
    prob = make_config("c1")
    x0 = x0_batch(prob.nx, 1, 1002, scale=20.0)[0]
    q, l, u = prob.instance(x0)
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp32", n_rho=8)
    sol.solve()
    res = sol.result()
    sol.close()
    assert res["status"] == rq.RQP_SOLVED
    assert_passes_fp64_test(prob.P, q, prob.A, res["x"], res["z"], res["y"], what="c1 fp32 x0 x 20")


def test_nonfinite_status(rq, c0):
    prob, x0 = c0
    q, l, u = prob.instance(x0[0])
    q = q.copy()
    q[3] = np.nan
    for prec in ("fp64", "fp32"):
        sol = rq.Solver(prob.P, q, prob.A, l, u, precision=prec)
        sol.solve()
        res = sol.result()
        sol.close()
        assert res["status"] == rq.RQP_NONFINITE and res["iterations"] == 25


def test_warm_start_and_update(rq, c0):
    prob, x0 = c0
    q, l, u = prob.instance(5.0 * x0[2])
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp64", n_rho=8)
    sol.solve()
    r1 = sol.result()
    assert r1["status"] == rq.RQP_SOLVED
    # warm start from the solution: converged at the first check (Sec. II-B warm starting)
    sol.warm_start(r1["x"], r1["y"], r1["rho_index"])
    sol.solve()
    r2 = sol.result()
    assert r2["status"] == rq.RQP_SOLVED and r2["iterations"] == 25
    ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(n_rho=8), warm=(r1["x"], r1["y"], r1["rho_index"]))
    assert ref.iterations == 25
    _compare(r2, ref, 1e-9)
    # new data through the host update, cold start again
    q2, l2, u2 = prob.instance(5.0 * x0[3])
    sol.update(q2, l2, u2)
    sol.solve()
    r3 = sol.result()
    ref3 = oracle.solve(prob.P, q2, prob.A, l2, u2, _oracle_settings(n_rho=8))
    assert r3["iterations"] == ref3.iterations and r3["rho_hist"] == ref3.rho_hist
    _compare(r3, ref3, 1e-9)
    sol.close()


def test_parametric_update_matches_oracle(rq, c0):
    import torch

    prob, x0s = c0
    q, l, u = prob.instance(x0s[0])
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp64", eps_abs=0.0, eps_rel=0.0, max_iter=40)
    sol.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    x0 = 5.0 * x0s[1]
    sol.update_x0_device(torch.tensor(x0, dtype=torch.float64, device="cuda"))
    sol.solve()
    res = sol.result()
    sol.close()
    q2, l2, u2 = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, x0)
    ref = oracle.solve(prob.P, q2, prob.A, l2, u2, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=40))
    _compare(res, ref, 1e-9)


def test_launch_shape_limits(rq):
    P, q, A, l, u = random_qp(120, 20, 40, seed=11)
    sol = rq.Solver(P, q, A, l, u, precision="fp32")
    assert sol.launch() == (15, 1024)  # plain solves: ceil(180 / 12.5) workgroups by default
    for bad in (1, 2, 181):  # at most 64 rows per workgroup, at least one row each
        with pytest.raises(rq.ReluQPError):
            sol.set_launch(bad)
    sol.set_launch(3)
    assert sol.launch()[0] == 3
    sol.set_launch(0)
    assert sol.launch()[0] == 15
    sol.close()


def test_setup_errors(rq):
    P, q, A, l, u = random_qp(10, 2, 3, seed=0)
    with pytest.raises(rq.ReluQPError) as e:
        rq.Solver(-P, q, A, l, u, precision="fp64")
    assert "RQP_ENOTPD" in str(e.value)
    with pytest.raises(rq.ReluQPError) as e:
        rq.Solver(P, q, A, u + 1.0, u, precision="fp64")
    assert "RQP_EINVAL" in str(e.value)
    Pa = P.copy()
    Pa[0, 1] += 1.0
    with pytest.raises(rq.ReluQPError):
        rq.Solver(Pa, q, A, l, u)


def test_abort(rq):
    import time

    P, q, A, l, u = random_qp(200, 10, 50, seed=5)
    sol = rq.Solver(P, q, A, l, u, precision="fp32", eps_abs=0.0, eps_rel=0.0, max_iter=2_000_000)
    sol.solve()
    time.sleep(0.05)
    sol.abort()
    res = sol.result()
    sol.close()
    assert res["status"] == rq.RQP_ABORTED
    assert 0 < res["iterations"] < 2_000_000 and res["iterations"] % 25 == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_x0_fuses_the_update(rq, c0, prec):
    """relu_qp_solve_x0 (update from x0 inside the solve launch) gives the bit-identical result
    of relu_qp_update_x0_device followed by relu_qp_solve, and matches the oracle."""
    import torch

    prob, x0 = c0
    xs = 5.0 * x0_batch(prob.nx, 3, 1200)
    q0, l0, u0 = prob.instance(xs[0])
    kw = dict(precision=prec, n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=75)
    a = rq.Solver(prob.P, q0, prob.A, l0, u0, **kw)
    b = rq.Solver(prob.P, q0, prob.A, l0, u0, **kw)
    for s in (a, b):
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    for i in range(1, 3):
        xd = torch.tensor(xs[i], dtype=torch.float64, device="cuda")
        a.solve_x0(xd)
        b.update_x0_device(xd)
        b.solve()
        ra, rb = a.result(), b.result()
        assert ra["rho_hist"] == rb["rho_hist"] and ra["iterations"] == rb["iterations"] == 75
        for name in ("x", "y", "z"):
            assert np.array_equal(ra[name], rb[name]), (prec, i, name)
        q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, xs[i])
        ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=75, n_rho=8),
                           rho_replay=ra["rho_hist"])
        _compare(ra, ref, TOL[prec])
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("chain", [False, True])
def test_solve_sequence_matches_separate_solves(rq, c0, prec, chain):
    """count solves in one launch (weights kept on chip between them) give the bit-identical
    results of the same solves launched one at a time, cold or warm-chained (each solve starts
    from the previous solution); the per-solve histories land at their own offsets."""
    import torch

    prob, _ = c0
    xs = 5.0 * x0_batch(prob.nx, 6, 1300)
    q0, l0, u0 = prob.instance(xs[0])
    kw = dict(precision=prec, n_rho=8, max_iter=400)
    seq = rq.Solver(prob.P, q0, prob.A, l0, u0, **kw)
    one = rq.Solver(prob.P, q0, prob.A, l0, u0, **kw)
    for s in (seq, one):
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        s.set_warm(chain)
    xd = torch.tensor(xs, dtype=torch.float64, device="cuda")
    out = seq.solve_sequence(xd)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "_result"}
    for i in range(len(xs)):
        one.solve_x0(xd[i:i + 1])
        r = one.result()
        assert res["status"][i] == r["status"] == rq.RQP_SOLVED, i
        assert res["iterations"][i] == r["iterations"] and res["rho_index"][i] == r["rho_index"], i
        nck = len(r["rho_hist"])
        assert res["rho_hist"][i][:nck].tolist() == r["rho_hist"], i
        np.testing.assert_array_equal(res["prim_res"][i][:nck], r["prim_res"])
        for name in ("x", "y", "z"):
            assert np.array_equal(res[name][i].astype(np.float64), r[name]), (prec, chain, i, name)
    # the chained solves also match the oracle's warm starts
    if chain and prec == "fp64":
        prev = None
        for i in range(3):
            q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, xs[i])
            ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(n_rho=8, max_iter=400), warm=prev)
            assert ref.iterations == res["iterations"][i]
            _compare({k: res[k][i] for k in ("x", "y", "z")}, ref, 1e-9)
            prev = (ref.x, ref.y, ref.rho_index)
    seq.close()
    one.close()


def test_smallest_problem_and_infinite_bounds(rq):
    """n = m = 1 (two layer rows: the single-workgroup kernel, and the persistent one on two
    workgroups), and a problem whose bounds are all infinite, where the fixed point is the
    closed form x = -P^-1 q."""
    P = np.array([[2.0]])
    q = np.array([1.0])
    A = np.array([[1.0]])
    for prec in ("fp64", "fp32"):
        for grid in (None, 2):
            res = _fixed_run(rq, P, q, A, np.array([-0.25]), np.array([0.25]), prec, 50, grid=grid)
            ref = oracle.solve(P, q, A, np.array([-0.25]), np.array([0.25]),
                               _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=50))
            _compare(res, ref, TOL[prec])
    rng = np.random.default_rng(3)
    M = rng.standard_normal((30, 30))
    P = M @ M.T / 30 + np.eye(30)
    q = rng.standard_normal(30)
    A = rng.standard_normal((12, 30))
    inf = np.full(12, np.inf)
    sol = rq.Solver(P, q, A, -inf, inf, precision="fp64", eps_abs=1e-9, eps_rel=1e-9, max_iter=4000)
    sol.solve()
    res = sol.result()
    sol.close()
    assert res["status"] == rq.RQP_SOLVED
    np.testing.assert_allclose(res["x"], -np.linalg.solve(P, q), rtol=0, atol=1e-6)


def test_wide_rows_streamed_fp32(rq):
    """L = 5200 (eight columns per lane, part of each block's rows streamed from memory every
    iteration) in FP32, 60 iterations against the oracle with the schedule replayed."""
    P, q, A, l, u = random_qp(2600, 100, 2500, seed=13)
    res = _fixed_run(rq, P, q, A, l, u, "fp32", 60, n_rho=8)
    ref = oracle.solve(P, q, A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=60, n_rho=8),
                       rho_replay=res["rho_hist"])
    _close(res["x"], ref.x, 1e-4, "x")
    _close(res["z"], ref.z, 1e-4, "z")
    # the iteration holds y_i / rho_i to FP32 precision: equality rows (rho_i = 1000 rho) are
    # compared at 1e-4 rho_i max(|z|, 1), the others at 1e-4 max(|y|, 1)
    eq = l == u
    dy = np.abs(res["y"] - ref.y)
    assert np.max(dy[~eq]) <= 1e-4 * max(np.max(np.abs(ref.y)), 1.0)
    rho_eq = max(admm.rho_grid(_oracle_settings(n_rho=8))[j] for j in res["rho_hist"] + [2]) * 1e3
    assert np.max(dy[eq]) <= 1e-4 * rho_eq * max(np.max(np.abs(ref.z)), 1.0)


def test_maximum_size_fp32(rq):
    """n + m = 8192, the largest problem the single-instance engine accepts (n = 4096, 96
    equality and 4000 inequality rows): 25 iterations and one check against the oracle with the
    schedule replayed, and one row past the limit rejected at setup."""
    P, q, A, l, u = random_qp(4096, 96, 4000, seed=17)
    res = _fixed_run(rq, P, q, A, l, u, "fp32", 25, n_rho=8)
    ref = oracle.solve(P, q, A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=25, n_rho=8),
                       rho_replay=res["rho_hist"])
    _close(res["x"], ref.x, 1e-4, "x")
    _close(res["z"], ref.z, 1e-4, "z")
    eq = l == u
    dy = np.abs(res["y"] - ref.y)
    assert np.max(dy[~eq]) <= 1e-4 * max(np.max(np.abs(ref.y)), 1.0)
    rho_eq = max(admm.rho_grid(_oracle_settings(n_rho=8))[j] for j in res["rho_hist"] + [2]) * 1e3
    assert np.max(dy[eq]) <= 1e-4 * rho_eq * max(np.max(np.abs(ref.z)), 1.0)
    A1 = np.vstack([A, A[:1]])
    with pytest.raises(rq.ReluQPError):
        rq.Solver(P, q, A1, np.append(l, l[0] - 1.0), np.append(u, u[0] + 1.0), precision="fp32")


def test_c2_humanoid_shape_fp32(rq):
    """Configuration 2 (n = 600 controls, m = 1800: control limits and condensed state limits),
    FP32: 100 fixed iterations against the oracle with the GPU's schedule replayed, and a solve
    to eps = 1e-3 that passes the FP64 residual test and lies near the oracle's solution."""
    prob = make_config("c2")
    x0 = x0_batch(prob.nx, 2, 1020, scale=3.0)  # scaled so that limits bind (1-2 % active rows)
    q, l, u = prob.instance(x0[0])
    res = _fixed_run(rq, prob.P, q, prob.A, l, u, "fp32", 100, n_rho=8)
    ref = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=0.0, eps_rel=0.0, max_iter=100, n_rho=8),
                       rho_replay=res["rho_hist"])
    _compare(res, ref, TOL["fp32"])
    q, l, u = prob.instance(x0[1])
    sol = rq.Solver(prob.P, q, prob.A, l, u, precision="fp32", n_rho=8)
    sol.solve()
    r = sol.result()
    sol.close()
    assert r["status"] == rq.RQP_SOLVED
    assert_passes_fp64_test(prob.P, q, prob.A, r["x"], r["z"], r["y"], what="c2 fp32")
    xs = oracle.solve(prob.P, q, prob.A, l, u, _oracle_settings(eps_abs=1e-10, eps_rel=1e-10, n_rho=8,
                                                                max_iter=40000)).x
    err = np.max(np.abs(r["x"] - xs)) / max(np.max(np.abs(xs)), 1.0)
    print(f"\nc2 FP32 solution error at eps=1e-3: {err:.2e} ({r['iterations']} iterations)")
    assert err < 5e-2
