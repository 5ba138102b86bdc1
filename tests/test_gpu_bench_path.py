"""The launch the benchmark times, against the FP64 oracle: relu_qp_solve_sequence (several
solves in one persistent launch, q, l, u formed in the kernel from each solve's x0) on the
persistent kernel's plain instantiation, at the benchmark's default grid, cold and
warm-chained (each solve starts from the previous solution, z = A x), with limits idle (x0
scale 1: every solve stops at the first check) and binding (scale 20: penalties switch).

Per solve: the sequence is bit-identical to the same solves launched one at a time
(relu_qp_solve_x0); x, z and y match the oracle fed q, l, u = (F x0, lo - E x0, hi - E x0)
(oracle.mpc_update) over the same iterations with the GPU's penalty schedule replayed, within
1e-4 (FP32) or 1e-9 (FP64) relative; chained solves are compared with the oracle's own warm
starts from its previous solution; every final solution passes the FP64 stopping test at
1.0 x eps when re-evaluated on the CPU. The FP64 case (n + m = 300) is above the
single-workgroup limit, so it runs the persistent kernel too (default and explicit grid).
"""

import numpy as np
import pytest

import oracle
from oracle import admm
from oracle.mpc_update import qp_vectors
from residual_check import assert_passes_fp64_test
from workloads import make_config, random_mpc, x0_batch

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}
SETTINGS = dict(n_rho=8, rho0=0.1, sigma=1e-6, alpha=1.6, eps_abs=1e-3, eps_rel=1e-3, max_iter=4000,
                check_interval=25)
_PROBS = {}
_CACHES = {}


@pytest.fixture(scope="module")
def rq():
    import paper_2311_18056_amd as rq

    rq.lib()
    return rq


def _prob(name):
    if name not in _PROBS:
        # c1: the benchmark's family; mpc300: nx = 15, nu = 5, N = 30 (n = m = 150)
        _PROBS[name] = make_config("c1") if name == "c1" else random_mpc(15, 5, 30, seed=77)
        _CACHES[name] = {}
    return _PROBS[name], _CACHES[name]


def _close(a, b, tol, what):
    err = np.max(np.abs(a - b))
    scale = max(np.max(np.abs(b)), 1.0)
    assert err <= tol * scale, f"{what}: |diff| = {err:.3e} > {tol:.1e} * {scale:.3e}"
    return err / scale


@pytest.mark.parametrize("name,prec,scale,chain,grid", [
    ("c1", "fp32", 1.0, False, None),
    ("c1", "fp32", 1.0, True, None),
    ("c1", "fp32", 20.0, False, None),
    ("c1", "fp32", 20.0, True, None),
    ("mpc300", "fp64", 5.0, False, None),
    ("mpc300", "fp64", 5.0, True, None),
    ("mpc300", "fp64", 5.0, True, 7),
])
def test_sequence_on_the_benchmark_launch(rq, name, prec, scale, chain, grid):
    import torch

    prob, cache = _prob(name)
    count = 4
    xs = x0_batch(prob.nx, count, 1000, scale=scale)  # the benchmark's x0 stream
    q0, l0, u0 = prob.instance(xs[0])
    seq = rq.Solver(prob.P, q0, prob.A, l0, u0, precision=prec, **SETTINGS)
    one = rq.Solver(prob.P, q0, prob.A, l0, u0, precision=prec, **SETTINGS)
    for s in (seq, one):
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        s.set_warm(chain)
        if grid is not None:
            s.set_launch(grid)
    L = prob.n + prob.m
    want = grid if grid is not None else (256 if name == "c1" else -(-L * 2 // 25))
    assert seq.launch() == (want, 1024), seq.launch()
    print(f"\n{name} {prec} x0 x {scale:g} chain={chain}: grid {seq.launch()[0]}", flush=True)
    xd = torch.tensor(xs, dtype=torch.float64, device="cuda")
    out = seq.solve_sequence(xd)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "_result"}

    prev = None
    for i in range(count):
        # the same solve launched alone (the previous one chained in the handle) is bit-identical
        one.solve_x0(xd[i:i + 1])
        r = one.result()
        it, st = int(res["iterations"][i]), int(res["status"][i])
        assert st == r["status"] == rq.RQP_SOLVED, (i, st)
        assert it == r["iterations"] and int(res["rho_index"][i]) == r["rho_index"], i
        nck = len(r["rho_hist"])
        assert res["rho_hist"][i][:nck].tolist() == r["rho_hist"], i
        for v in ("x", "y", "z"):
            assert np.array_equal(res[v][i].astype(np.float64), r[v]), (i, v)

        # the oracle over the same iterations, the GPU's schedule replayed, from its own warm start
        q, l, u = qp_vectors(prob.F, prob.E, prob.lo, prob.hi, xs[i])
        s = admm.Settings(n_rho=8, eps_abs=0.0, eps_rel=0.0, max_iter=it)
        ref = oracle.solve(prob.P, q, prob.A, l, u, s, rho_replay=r["rho_hist"], warm=prev, cache=cache)
        assert ref.rho_index == r["rho_index"]
        errs = [_close(r[v], getattr(ref, v), TOL[prec], f"solve {i} {v}") for v in ("x", "z", "y")]
        worst = assert_passes_fp64_test(prob.P, q, prob.A, r["x"], r["z"], r["y"], what=f"solve {i}")
        print(f"solve {i}: {it} iterations, penalties {r['rho_hist']}, max rel diff {max(errs):.2e}, "
              f"FP64 test ratio {worst:.4f}", flush=True)
        if prec == "fp64":
            # FP64 takes the oracle's own decisions: same stopping check and schedule
            own = oracle.solve(prob.P, q, prob.A, l, u, admm.Settings(**{k: v for k, v in SETTINGS.items()}),
                               warm=prev, cache=cache)
            assert own.iterations == it and own.rho_hist == r["rho_hist"], (own.iterations, own.rho_hist)
        prev = (ref.x, ref.y, ref.rho_index) if chain else None
    seq.close()
    one.close()
