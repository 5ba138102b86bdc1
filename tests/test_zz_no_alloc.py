"""relu_qp_solve_x0_noalloc (the launch's scratch in the library's static device array, no
allocation) against relu_qp_solve_x0 on the same handle state and x0: every output
bit-identical, on two calls in a row, the second with a smaller problem (the scratch keeps the
first call's words; monotone tags keep them from matching), and the small-problem kernel too.
Through the C ABI; runs alone in a fresh process or after the other GPU tests."""

import numpy as np
import pytest

from workloads import make_config, random_mpc, x0_batch

pytestmark = pytest.mark.gpu

SETTINGS = dict(n_rho=8, rho0=0.1, sigma=1e-6, alpha=1.6, eps_abs=1e-3, eps_rel=1e-3, max_iter=4000,
                check_interval=25)


@pytest.fixture(scope="module")
def rq():
    import paper_2311_18056_amd as rq

    rq.lib()
    return rq


def _pair(rq, prob, prec, chain):
    q, l, u = prob.instance(np.zeros(prob.nx))
    out = []
    for _ in range(2):
        s = rq.Solver(prob.P, q, prob.A, l, u, precision=prec, **SETTINGS)
        s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
        s.set_warm(chain)
        out.append(s)
    return out


def _same(a, b, what):
    assert a["status"] == b["status"] and a["iterations"] == b["iterations"], what
    assert a["rho_index"] == b["rho_index"] and a["rho_hist"] == b["rho_hist"], what
    assert np.array_equal(a["prim_res"], b["prim_res"]) and np.array_equal(a["dual_res"], b["dual_res"]), what
    for v in ("x", "y", "z"):
        assert np.array_equal(a[v], b[v]), (what, v)


def test_noalloc_matches_solve_x0_two_calls_second_smaller(rq):
    import torch

    cases = [
        ("c1 FP32 (n + m = 3200, persistent grid)", make_config("c1"), "fp32", 20.0),
        ("n + m = 300 FP64 (persistent grid)", random_mpc(15, 5, 30, seed=77), "fp64", 5.0),
        ("c0 FP64 (n + m = 40, one workgroup)", make_config("c0"), "fp64", 5.0),
    ]
    for name, prob, prec, scale in cases:
        print(f"\n{name}", flush=True)
        for chain in (False, True):
            ref, noalloc = _pair(rq, prob, prec, chain)
            xs = x0_batch(prob.nx, 2, 1000, scale=scale)
            for i in range(2):  # a second call on the same handles (chained: warm from the first)
                xd = torch.tensor(xs[i:i + 1], dtype=torch.float64, device="cuda")
                ref.solve_x0(xd)
                noalloc.solve_x0_noalloc(xd)
                a, b = ref.result(), noalloc.result()
                assert a["status"] == rq.RQP_SOLVED, (name, chain, i)
                _same(a, b, (name, chain, i))
                print(f"  chain={chain} call {i}: {a['iterations']} iterations, identical", flush=True)
            ref.close()
            noalloc.close()


def test_noalloc_rejects_the_batched_engine(rq):
    prob = make_config("c0")
    q, l, u = prob.instance(np.zeros(prob.nx))
    B = 4
    s = rq.Solver(prob.P, np.tile(q, (B, 1)), prob.A, np.tile(l, (B, 1)), np.tile(u, (B, 1)), precision="fp32",
                  engine="batch", **SETTINGS)
    s.set_parametric(prob.F, prob.E, prob.lo, prob.hi)
    import torch

    with pytest.raises(rq.ReluQPError) as e:
        s.solve_x0_noalloc(torch.zeros(B, prob.nx, dtype=torch.float64, device="cuda"))
    assert "RQP_ESTATE" in str(e.value)
    s.close()
