"""ctypes declarations of the C ABI in ``include/relu_qp.h`` (argument marshalling only).

The shared library is built in-tree by ``paper_2311_18056_amd.build``. Loading it never falls
back to anything else: if it is missing the import of this module's ``lib()`` raises.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librelu_qp.so")

RQP_OK, RQP_EINVAL, RQP_ENOMEM, RQP_EHIP, RQP_ENOTPD, RQP_ESTATE = 0, -1, -2, -3, -4, -5
RQP_RUNNING, RQP_SOLVED, RQP_MAX_ITER, RQP_NONFINITE, RQP_ABORTED, RQP_INTERNAL, RQP_IDLE = 0, 1, 2, 3, 4, 5, 6
RQP_FP64, RQP_FP32, RQP_BF16X3 = 0, 1, 2
RQP_ENGINE_AUTO, RQP_ENGINE_SINGLE, RQP_ENGINE_BATCH = 0, 1, 2

ERROR_NAMES = {
    RQP_EINVAL: "RQP_EINVAL",
    RQP_ENOMEM: "RQP_ENOMEM",
    RQP_EHIP: "RQP_EHIP",
    RQP_ENOTPD: "RQP_ENOTPD",
    RQP_ESTATE: "RQP_ESTATE",
}

# every symbol the header declares
EXPORTS = [
    "relu_qp_default_settings",
    "relu_qp_setup",
    "relu_qp_update",
    "relu_qp_update_device",
    "relu_qp_set_parametric",
    "relu_qp_update_x0_device",
    "relu_qp_warm_start",
    "relu_qp_set_warm",
    "relu_qp_solve",
    "relu_qp_solve_x0",
    "relu_qp_solve_x0_noalloc",
    "relu_qp_solve_sequence",
    "relu_qp_load_slots",
    "relu_qp_load_slots_x0",
    "relu_qp_admit",
    "relu_qp_step",
    "relu_qp_get_tile",
    "relu_qp_set_tile",
    "relu_qp_device_bytes",
    "relu_qp_closed_loop",
    "relu_qp_solve_paper_form",
    "relu_qp_offload",
    "relu_qp_restore",
    "relu_qp_footprint",
    "relu_qp_abort",
    "relu_qp_max_checks",
    "relu_qp_get_rho_grid",
    "relu_qp_set_launch",
    "relu_qp_get_launch",
    "relu_qp_cleanup",
    "relu_qp_last_error",
]


class Settings(Structure):
    _fields_ = [
        ("sigma", c_double),
        ("alpha", c_double),
        ("rho0", c_double),
        ("n_rho", c_int),
        ("rho_min", c_double),
        ("rho_max", c_double),
        ("rho_eq_scale", c_double),
        ("eps_abs", c_double),
        ("eps_rel", c_double),
        ("max_iter", c_int),
        ("check_interval", c_int),
        ("precision", c_int),
        ("batch", c_int),
        ("engine", c_int),
        ("scaling", c_int),
    ]


class Result(Structure):
    _fields_ = [
        ("x", c_void_p),
        ("y", c_void_p),
        ("z", c_void_p),
        ("iterations", c_void_p),
        ("status", c_void_p),
        ("rho_index", c_void_p),
        ("rho_hist", c_void_p),
        ("prim_res", c_void_p),
        ("dual_res", c_void_p),
    ]


class ReluQPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_LIB = None
_dp = POINTER(c_double)


def lib():
    """The loaded library (loaded once). Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2311_18056_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    h = c_void_p
    L.relu_qp_default_settings.argtypes = [POINTER(Settings)]
    L.relu_qp_default_settings.restype = None
    L.relu_qp_setup.argtypes = [POINTER(h), c_int, c_int, _dp, _dp, _dp, _dp, _dp, POINTER(Settings), c_void_p]
    L.relu_qp_update.argtypes = [h, _dp, _dp, _dp]
    L.relu_qp_update_device.argtypes = [h, c_void_p, c_void_p, c_void_p, c_void_p]
    L.relu_qp_set_parametric.argtypes = [h, c_int, _dp, _dp, _dp, _dp]
    L.relu_qp_update_x0_device.argtypes = [h, c_void_p, c_void_p]
    L.relu_qp_warm_start.argtypes = [h, _dp, _dp, c_int]
    L.relu_qp_set_warm.argtypes = [h, c_int]
    L.relu_qp_solve.argtypes = [h, c_void_p, POINTER(Result)]
    L.relu_qp_solve_x0.argtypes = [h, c_void_p, c_void_p, POINTER(Result)]
    L.relu_qp_solve_x0_noalloc.argtypes = [h, c_void_p, c_void_p, POINTER(Result)]
    L.relu_qp_solve_sequence.argtypes = [h, c_void_p, c_int, c_void_p, POINTER(Result)]
    _ip = POINTER(c_int)
    L.relu_qp_load_slots.argtypes = [h, _ip, c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.relu_qp_load_slots_x0.argtypes = [h, _ip, c_int, c_void_p, c_void_p]
    L.relu_qp_admit.argtypes = [h, _ip, c_int, c_int, c_int, c_int, c_void_p]
    L.relu_qp_step.argtypes = [h, c_int, c_void_p, POINTER(Result)]
    L.relu_qp_get_tile.argtypes = [h, POINTER(c_int), POINTER(c_double)]
    L.relu_qp_set_tile.argtypes = [h, c_int]
    L.relu_qp_device_bytes.argtypes = [h, POINTER(c_size_t)]
    L.relu_qp_solve_paper_form.argtypes = [h, c_int, c_void_p, POINTER(Result)]
    L.relu_qp_offload.argtypes = [h]
    L.relu_qp_restore.argtypes = [h]
    L.relu_qp_closed_loop.argtypes = [h, c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                                      POINTER(Result)]
    L.relu_qp_footprint.argtypes = [c_int, c_int, POINTER(Settings), c_int, POINTER(c_size_t), POINTER(c_size_t)]
    L.relu_qp_abort.argtypes = [h]
    L.relu_qp_max_checks.argtypes = [h]
    L.relu_qp_get_rho_grid.argtypes = [h, _dp, POINTER(c_int)]
    L.relu_qp_set_launch.argtypes = [h, c_int]
    L.relu_qp_get_launch.argtypes = [h, POINTER(c_int), POINTER(c_int)]
    L.relu_qp_cleanup.argtypes = [h]
    L.relu_qp_last_error.argtypes = []
    L.relu_qp_last_error.restype = c_char_p
    for name in EXPORTS:
        if name not in ("relu_qp_default_settings", "relu_qp_last_error"):
            getattr(L, name).restype = c_int
    _LIB = L
    return L


def check(rc: int) -> int:
    if rc < 0:
        raise ReluQPError(rc, lib().relu_qp_last_error().decode())
    return rc
