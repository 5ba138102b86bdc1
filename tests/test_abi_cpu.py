"""Host-side checks of the C ABI (no GPU): the library loads and exports every declared symbol,
and the header and the binding agree on the settings defaults."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "relu_qp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(relu_qp_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_list_the_same_symbols():
    from paper_2311_18056_amd._lib import EXPORTS

    assert sorted(EXPORTS) == _declared_functions()


def test_library_exports_every_symbol():
    import paper_2311_18056_amd as rq

    lib = rq.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_default_settings():
    import paper_2311_18056_amd as rq

    s = rq.default_settings()
    assert (s.sigma, s.alpha, s.rho0, s.n_rho) == (1e-6, 1.6, 0.1, 1)
    assert (s.rho_min, s.rho_max, s.rho_eq_scale) == (1e-3, 1e3, 1e3)
    assert (s.eps_abs, s.eps_rel, s.max_iter, s.check_interval) == (1e-3, 1e-3, 4000, 25)
    assert s.batch == 1 and s.scaling == 0
    with pytest.raises(AttributeError):
        rq.default_settings(no_such_field=1)


def test_null_handle_is_rejected_without_a_gpu():
    import ctypes

    import paper_2311_18056_amd as rq

    lib = rq.lib()
    assert lib.relu_qp_cleanup(None) == 0
    assert lib.relu_qp_abort(None) == rq._lib.RQP_ESTATE
    assert b"NULL handle" in lib.relu_qp_last_error()
    assert lib.relu_qp_solve(None, None, None) == rq._lib.RQP_ESTATE
    s = rq.default_settings(alpha=2.5)
    h = ctypes.c_void_p()
    z = (ctypes.c_double * 4)()
    rc = lib.relu_qp_setup(ctypes.byref(h), 2, 2, z, z, z, z, z, ctypes.byref(s), None)
    assert rc == rq._lib.RQP_EINVAL and h.value is None
    assert b"alpha" in lib.relu_qp_last_error()


def test_serving_calls_reject_a_null_handle():
    import paper_2311_18056_amd as rq

    lib = rq.lib()
    E = rq._lib.RQP_ESTATE
    assert lib.relu_qp_load_slots(None, None, 0, None, None, None, None) == E
    assert lib.relu_qp_load_slots_x0(None, None, 0, None, None) == E
    assert lib.relu_qp_admit(None, None, 0, -1, 0, 0, None) == E
    assert lib.relu_qp_step(None, 1, None, None) == E
    assert lib.relu_qp_closed_loop(None, None, 1, None, None, 1, None, None, None, None) == E


def test_settings_rules_for_engines():
    import ctypes

    import paper_2311_18056_amd as rq

    lib = rq.lib()
    h = ctypes.c_void_p()
    z = (ctypes.c_double * 4)()
    for kw, word in ((dict(precision="fp64", engine="batch"), b"FP32 or BF16X3"),
                     (dict(precision="bf16x3", engine="single"), b"batched engine"),
                     (dict(batch=2, engine="single"), b"batch == 1")):
        s = rq.default_settings(**kw)
        assert lib.relu_qp_setup(ctypes.byref(h), 2, 2, z, z, z, z, z, ctypes.byref(s), None) == rq._lib.RQP_EINVAL
        assert word in lib.relu_qp_last_error(), kw


def _setup_rc(n, m, P, q, A, l, u, **settings):
    """relu_qp_setup's return code and message for host arrays (validation runs before any
    device call, so no GPU is needed for the rejected cases)."""
    import ctypes

    import numpy as np

    import paper_2311_18056_amd as rq

    lib = rq.lib()
    s = rq.default_settings(**settings)
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)).ravel() for a in (P, q, A, l, u)]
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
    h = ctypes.c_void_p()
    rc = lib.relu_qp_setup(ctypes.byref(h), n, m, *ptrs, ctypes.byref(s), None)
    assert h.value is None
    return rc, lib.relu_qp_last_error().decode()


def test_setup_rejects_bad_problems():
    import numpy as np

    import paper_2311_18056_amd as rq

    E = rq._lib.RQP_EINVAL
    P, q, A = np.eye(2), np.zeros(2), np.eye(2)
    l, u = -np.ones(2), np.ones(2)
    cases = [
        ((0, 2, P, q, A, l, u), "n >= 1"),
        ((2, 0, P, q, A, l, u), "m >= 1"),
        ((2, 2, [[1, 0.5], [0.4, 1]], q, A, l, u), "symmetric"),
        ((2, 2, [[1, np.inf], [np.inf, 1]], q, A, l, u), "non-finite"),
        ((2, 2, P, q, [[1, np.nan], [0, 1]], l, u), "A has a non-finite"),
        ((2, 2, P, q, A, [2.0, -1.0], u), "l[0] > u[0]"),
        ((2, 2, P, q, A, [np.nan, -1.0], u), "NaN"),
        ((2, 2, P, q, A, [np.inf, -1.0], [np.inf, 1.0]), "empty box"),
        ((5000, 4000, np.eye(1), q, A, l, u), "exceeds"),
    ]
    for args, word in cases:
        rc, msg = _setup_rc(*args)
        assert rc == E and word in msg, (word, rc, msg)


def test_setup_rejects_bad_settings():
    import numpy as np

    import paper_2311_18056_amd as rq

    E = rq._lib.RQP_EINVAL
    P, q, A = np.eye(2), np.zeros(2), np.eye(2)
    l, u = -np.ones(2), np.ones(2)
    for kw, word in ((dict(sigma=0.0), "sigma"), (dict(alpha=0.0), "alpha"), (dict(n_rho=0), "n_rho"),
                     (dict(n_rho=65), "n_rho"), (dict(n_rho=8, rho_min=1.0, rho_max=0.5), "rho_min"),
                     (dict(eps_abs=-1.0), "eps_abs"), (dict(max_iter=0), "max_iter"),
                     (dict(check_interval=0), "check_interval"), (dict(precision=7), "precision"),
                     (dict(engine=9), "engine"), (dict(batch=0), "batch"), (dict(rho_eq_scale=0.0), "rho_eq_scale"),
                     (dict(scaling=-1), "scaling"), (dict(scaling=101), "scaling")):
        rc, msg = _setup_rc(2, 2, P, q, A, l, u, **kw)
        assert rc == E and word in msg, (kw, rc, msg)


def test_batched_setup_rejects_mixed_equality_patterns():
    import numpy as np

    import paper_2311_18056_amd as rq

    P, A = np.eye(2), np.eye(2)
    q = np.zeros((2, 2))
    l = np.array([[0.0, -1.0], [-1.0, -1.0]])
    u = np.array([[0.0, 1.0], [1.0, 1.0]])
    rc, msg = _setup_rc(2, 2, P, q, A, l, u, batch=2, precision="fp32")
    assert rc == rq._lib.RQP_EINVAL and "equality-row pattern" in msg


def test_handles_close_before_interpreter_shutdown():
    """Open handles are closed by an exit hook (while the HIP runtime is alive); a finaliser that
    runs during interpreter shutdown makes no library call."""
    import atexit  # noqa: F401
    import sys

    from paper_2311_18056_amd import solver

    assert solver.open_handles() == 0
    s = solver.Solver.__new__(solver.Solver)  # never set up: no handle
    s._h = solver.c_void_p()
    solver._OPEN.add(s)
    assert solver.open_handles() == 1
    solver.close_all()  # closing a handle-less solver makes no library call
    assert solver.open_handles() == 0
    assert not sys.is_finalizing()
