"""Python face of the C ABI: a QP handle whose results live in torch device tensors.

Every step of the solve runs in the HIP library; this module only marshals arguments. torch
provides the device memory of the result buffers and the stream.
"""

from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from ctypes import POINTER, byref, c_double, c_int, c_size_t, c_void_p

import numpy as np
import torch

from . import _lib
from ._lib import (RQP_BF16X3, RQP_ENGINE_AUTO, RQP_ENGINE_BATCH, RQP_ENGINE_SINGLE, RQP_FP32, RQP_FP64, Result,
                   Settings, check, lib)

STATUS_NAMES = {0: "running", 1: "solved", 2: "max_iter", 3: "nonfinite", 4: "aborted", 5: "internal", 6: "idle"}


# Handles still open. They are closed by an exit hook, which runs before the interpreter tears
# down its modules and while the HIP runtime (and a profiler attached to it) is still alive; a
# handle freed later, from a finaliser during interpreter shutdown, would call into a runtime
# that may already be gone.
_OPEN = weakref.WeakSet()


@atexit.register
def close_all():
    """Close every handle that is still open (also run at interpreter exit)."""
    for s in list(_OPEN):
        s.close()


def open_handles() -> int:
    return len(_OPEN)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _stream_handle(stream) -> c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def default_settings(**overrides) -> Settings:
    s = Settings()
    lib().relu_qp_default_settings(byref(s))
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": RQP_FP64, "fp32": RQP_FP32, "bf16x3": RQP_BF16X3}[v]
        if k == "engine" and isinstance(v, str):
            v = {"auto": RQP_ENGINE_AUTO, "single": RQP_ENGINE_SINGLE, "batch": RQP_ENGINE_BATCH}[v]
        if not hasattr(s, k):
            raise AttributeError(k)
        setattr(s, k, v)
    return s


def _result_bytes(n: int, m: int, batch: int, fp64: bool, max_checks: int) -> int:
    """Device bytes of a Solver's result tensors (x, y, z, counters, per-check histories)."""
    es = 8 if fp64 else 4
    return batch * ((n + 2 * m) * es + 3 * 4 + max_checks * (4 + 8 + 8))


def footprint(n: int, m: int, nx: int = 0, **settings) -> dict:
    """Device bytes a ``Solver`` of this size holds once set up (plus F, E, lo, hi when nx > 0):
    ``resident`` = the library's allocations + the result tensors; ``setup_extra`` = the FP64
    workspace the setup holds on top of that while it factors. No device call."""
    s = default_settings(**settings)
    lib_bytes, extra = c_size_t(), c_size_t()
    check(lib().relu_qp_footprint(int(n), int(m), byref(s), int(nx), byref(lib_bytes), byref(extra)))
    ci = max(int(s.check_interval), 1)
    max_checks = -(-int(s.max_iter) // ci)
    res = _result_bytes(n, m, int(s.batch), s.precision == RQP_FP64, max_checks)
    return {"resident": lib_bytes.value + res, "library": lib_bytes.value, "results": res,
            "setup_extra": extra.value}


class Solver:
    """One QP family (fixed P and A) with its device-resident layer weights.

    Parameters follow ``relu_qp_settings``; ``precision`` is "fp64" or "fp32".
    """

    def __init__(self, P, q, A, l, u, *, device="cuda:0", stream=None, **settings):
        """q: (n,) or (batch, n); l, u: (m,) or (batch, m). ``batch`` defaults to the leading
        dimension of q."""
        L = lib()
        P = _f64(P)
        n = P.shape[0]
        A = _f64(A)
        m = A.shape[0]
        q = _f64(q)
        batch = 1 if q.ndim == 1 else q.shape[0]
        settings.setdefault("batch", batch)
        if settings["batch"] != batch:
            raise ValueError("batch must match the leading dimension of q")
        q = _f64(q, (n,) if batch == 1 and q.ndim == 1 else (batch, n))
        l = _f64(l, (m,) if batch == 1 and np.ndim(l) == 1 else (batch, m))
        u = _f64(u, (m,) if batch == 1 and np.ndim(u) == 1 else (batch, m))
        if P.shape != (n, n) or A.shape != (m, n):
            raise ValueError("P must be n x n and A m x n")
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.settings = default_settings(**settings)
        self.n, self.m, self.batch = n, m, batch
        self._h = c_void_p()
        check(L.relu_qp_setup(byref(self._h), n, m, _ptr(P), _ptr(q), _ptr(A), _ptr(l), _ptr(u),
                              byref(self.settings), _stream_handle(stream)))
        _OPEN.add(self)
        self.max_checks = check(L.relu_qp_max_checks(self._h))
        self.fp64 = self.settings.precision == RQP_FP64
        self.dtype = torch.float64 if self.fp64 else torch.float32
        dev, B = self.device, batch
        self.x = torch.zeros(B, n, dtype=self.dtype, device=dev)
        self.y = torch.zeros(B, m, dtype=self.dtype, device=dev)
        self.z = torch.zeros(B, m, dtype=self.dtype, device=dev)
        self.iterations = torch.zeros(B, dtype=torch.int32, device=dev)
        self.status = torch.zeros(B, dtype=torch.int32, device=dev)
        self.rho_index = torch.zeros(B, dtype=torch.int32, device=dev)
        self.rho_hist = torch.full((B, self.max_checks), -1, dtype=torch.int32, device=dev)
        self.prim_res = torch.zeros(B, self.max_checks, dtype=torch.float64, device=dev)
        self.dual_res = torch.zeros(B, self.max_checks, dtype=torch.float64, device=dev)
        self._res = Result(
            self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(), self.iterations.data_ptr(),
            self.status.data_ptr(), self.rho_index.data_ptr(), self.rho_hist.data_ptr(),
            self.prim_res.data_ptr(), self.dual_res.data_ptr(),
        )

    # ------------------------------------------------------------------ online stage
    def update(self, q=None, l=None, u=None):
        n, m, B = self.n, self.m, self.batch
        args = [None if v is None else _f64(v).reshape(B * s) for v, s in ((q, n), (l, m), (u, m))]
        self._keep = args
        check(lib().relu_qp_update(self._h, *[None if a is None else _ptr(a) for a in args]))

    def update_device(self, q=None, l=None, u=None, stream=None):
        ptrs = []
        for v in (q, l, u):
            if v is None:
                ptrs.append(None)
            else:
                if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous():
                    raise ValueError("device updates take contiguous float64 cuda tensors")
                ptrs.append(c_void_p(v.data_ptr()))
        check(lib().relu_qp_update_device(self._h, *ptrs, _stream_handle(stream)))

    def set_parametric(self, F, E, lo, hi):
        F = _f64(F)
        nx = F.shape[1]
        E, lo, hi = _f64(E, (self.m, nx)), _f64(lo, (self.m,)), _f64(hi, (self.m,))
        check(lib().relu_qp_set_parametric(self._h, nx, _ptr(F), _ptr(E), _ptr(lo), _ptr(hi)))
        self.nx = nx

    def update_x0_device(self, x0: torch.Tensor, stream=None):
        if x0.dtype != torch.float64 or not x0.is_cuda or not x0.is_contiguous():
            raise ValueError("x0 must be a contiguous float64 cuda tensor")
        check(lib().relu_qp_update_x0_device(self._h, c_void_p(x0.data_ptr()), _stream_handle(stream)))

    def warm_start(self, x, y, rho_index: int):
        x, y = _f64(x).reshape(self.batch * self.n), _f64(y).reshape(self.batch * self.m)
        check(lib().relu_qp_warm_start(self._h, _ptr(x), _ptr(y), int(rho_index)))

    def set_warm(self, enabled: bool):
        check(lib().relu_qp_set_warm(self._h, 1 if enabled else 0))

    def solve(self, stream=None, out: Result | None = None):
        """Launch the whole online loop (asynchronous on the stream). ``out`` optionally names
        other device result buffers (a ``Result`` from ``result_slots``)."""
        check(lib().relu_qp_solve(self._h, _stream_handle(stream), byref(out if out is not None else self._res)))

    def solve_x0(self, x0: torch.Tensor, stream=None, out: Result | None = None):
        """Update q, l, u from initial states x0 (float64 cuda, batch x nx) and solve; one launch
        on the single-instance engine."""
        if x0.dtype != torch.float64 or not x0.is_cuda or not x0.is_contiguous():
            raise ValueError("x0 must be a contiguous float64 cuda tensor")
        check(lib().relu_qp_solve_x0(self._h, c_void_p(x0.data_ptr()), _stream_handle(stream),
                                     byref(out if out is not None else self._res)))

    def solve_x0_noalloc(self, x0: torch.Tensor, stream=None, out: Result | None = None):
        """solve_x0 with the launch's scratch in the library's static device array: the call
        allocates nothing (calls that overlap on one GPU race)."""
        if x0.dtype != torch.float64 or not x0.is_cuda or not x0.is_contiguous():
            raise ValueError("x0 must be a contiguous float64 cuda tensor")
        check(lib().relu_qp_solve_x0_noalloc(self._h, c_void_p(x0.data_ptr()), _stream_handle(stream),
                                             byref(out if out is not None else self._res)))

    def solve_sequence(self, x0s: torch.Tensor, stream=None, out=None):
        """len(x0s) solves in one launch of the single-instance engine, each from its own x0
        (float64 cuda, count x nx). Results go to ``out`` (a dict from ``sequence_slots``) or to
        new tensors, returned as that dict."""
        if x0s.dtype != torch.float64 or not x0s.is_cuda or not x0s.is_contiguous() or x0s.dim() != 2:
            raise ValueError("x0s must be a contiguous (count, nx) float64 cuda tensor")
        count = x0s.shape[0]
        if out is None:
            out = self.sequence_slots(count)
        check(lib().relu_qp_solve_sequence(self._h, c_void_p(x0s.data_ptr()), count, _stream_handle(stream),
                                           byref(out["_result"])))
        return out

    def solve_paper_form(self, iters: int, stream=None, out: Result | None = None):
        """``iters`` layers of the paper's literal form v <- clamp(W v + b) from v = 0 (alpha = 1,
        fixed penalty); x, z and the lagged dual go to the result tensors."""
        check(lib().relu_qp_solve_paper_form(self._h, int(iters), _stream_handle(stream),
                                             byref(out if out is not None else self._res)))

    def closed_loop(self, x0: torch.Tensor, steps: int, Ad: torch.Tensor, Bd: torch.Tensor, nu: int, stream=None,
                    out=None):
        """``steps`` MPC steps in one launch: each runs ``max_iter`` warm-started iterations from
        the plant state, applies the first stage's control and steps the plant x <- Ad x + Bd u
        on the device. x0 (nx), Ad (nx, nx), Bd (nx, nu): float64 cuda. Returns the dict of
        ``sequence_slots(steps)`` with ``traj_x`` (steps + 1, nx) and ``traj_u`` (steps, nu)."""
        for t in (x0, Ad, Bd):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("x0, Ad and Bd must be contiguous float64 cuda tensors")
        nx = x0.numel()
        if Ad.shape != (nx, nx) or Bd.shape != (nx, nu):
            raise ValueError("Ad must be (nx, nx) and Bd (nx, nu)")
        if out is None:
            out = self.sequence_slots(steps)
            out["traj_x"] = torch.zeros(steps + 1, nx, dtype=torch.float64, device=self.device)
            out["traj_u"] = torch.zeros(steps, nu, dtype=torch.float64, device=self.device)
        check(lib().relu_qp_closed_loop(self._h, c_void_p(x0.data_ptr()), int(steps), c_void_p(Ad.data_ptr()),
                                        c_void_p(Bd.data_ptr()), int(nu), c_void_p(out["traj_x"].data_ptr()),
                                        c_void_p(out["traj_u"].data_ptr()), _stream_handle(stream),
                                        byref(out["_result"])))
        return out

    def sequence_slots(self, count: int) -> dict:
        """Device result tensors for ``count`` solves of one sequence launch."""
        dev = self.device
        t = dict(
            x=torch.zeros(count, self.n, dtype=self.dtype, device=dev),
            y=torch.zeros(count, self.m, dtype=self.dtype, device=dev),
            z=torch.zeros(count, self.m, dtype=self.dtype, device=dev),
            iterations=torch.zeros(count, dtype=torch.int32, device=dev),
            status=torch.zeros(count, dtype=torch.int32, device=dev),
            rho_index=torch.zeros(count, dtype=torch.int32, device=dev),
            rho_hist=torch.full((count, self.max_checks), -1, dtype=torch.int32, device=dev),
            prim_res=torch.zeros(count, self.max_checks, dtype=torch.float64, device=dev),
            dual_res=torch.zeros(count, self.max_checks, dtype=torch.float64, device=dev),
        )
        t["_result"] = Result(t["x"].data_ptr(), t["y"].data_ptr(), t["z"].data_ptr(), t["iterations"].data_ptr(),
                              t["status"].data_ptr(), t["rho_index"].data_ptr(), t["rho_hist"].data_ptr(),
                              t["prim_res"].data_ptr(), t["dual_res"].data_ptr())
        return t

    # ------------------------------------------------------------------ serving (batched engine)
    @staticmethod
    def _slot_array(slots):
        arr = (c_int * len(slots))(*[int(s) for s in slots])
        return arr, len(slots)

    @staticmethod
    def _dev_f64(t):
        if t is None:
            return None
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("slot data are contiguous float64 cuda tensors")
        return c_void_p(t.data_ptr())

    def load_slots(self, slots, q=None, l=None, u=None, stream=None):
        """q (len(slots), n), l, u (len(slots), m): float64 cuda tensors; None keeps a vector."""
        arr, k = self._slot_array(slots)
        check(lib().relu_qp_load_slots(self._h, arr, k, self._dev_f64(q), self._dev_f64(l), self._dev_f64(u),
                                       _stream_handle(stream)))

    def load_slots_x0(self, slots, x0: torch.Tensor, stream=None):
        """x0: (len(slots), nx) float64 cuda tensor; needs ``set_parametric``."""
        arr, k = self._slot_array(slots)
        check(lib().relu_qp_load_slots_x0(self._h, arr, k, self._dev_f64(x0), _stream_handle(stream)))

    def admit(self, slots, src_slot: int = -1, shift_x: int = 0, shift_y: int = 0, stream=None):
        """Start the listed slots at the next ``step``: cold (src_slot = -1) or warm from slot
        src_slot's x and y shifted by shift_x / shift_y entries, with z = A x."""
        arr, k = self._slot_array(slots)
        check(lib().relu_qp_admit(self._h, arr, k, int(src_slot), int(shift_x), int(shift_y),
                                  _stream_handle(stream)))

    def step(self, n_checks: int = 1, stream=None):
        """Run up to n_checks * check_interval iterations of every running or admitted slot
        (asynchronous); results of all slots land in this object's tensors."""
        check(lib().relu_qp_step(self._h, int(n_checks), _stream_handle(stream), byref(self._res)))

    def result_slots(self, count: int):
        """Device buffers for ``count`` solves (one slot each) and their ``Result`` structs.

        Returns (tensors, results): tensors is a dict of batched tensors (x: count x n, ...).
        """
        dev = self.device
        t = dict(
            x=torch.zeros(count, self.n, dtype=self.dtype, device=dev),
            y=torch.zeros(count, self.m, dtype=self.dtype, device=dev),
            z=torch.zeros(count, self.m, dtype=self.dtype, device=dev),
            iterations=torch.zeros(count, dtype=torch.int32, device=dev),
            status=torch.zeros(count, dtype=torch.int32, device=dev),
            rho_index=torch.zeros(count, dtype=torch.int32, device=dev),
        )
        res = [
            Result(t["x"][i].data_ptr(), t["y"][i].data_ptr(), t["z"][i].data_ptr(), t["iterations"][i].data_ptr(),
                   t["status"][i].data_ptr(), t["rho_index"][i].data_ptr(), None, None, None)
            for i in range(count)
        ]
        return t, res

    def tile(self):
        """(tile rows in use, {128: us/iter, 64: us/iter, 256: us/iter} from the autotuner) of a
        batched handle."""
        t = c_int()
        us = (c_double * 3)()
        check(lib().relu_qp_get_tile(self._h, byref(t), us))
        return t.value, {128: us[0], 64: us[1], 256: us[2]}

    def offload(self):
        """Move the handle's device memory to pinned host memory (the result tensors stay)."""
        check(lib().relu_qp_offload(self._h))

    def restore(self):
        """Bring an offloaded handle back to the device, exactly as it was."""
        check(lib().relu_qp_restore(self._h))

    def device_bytes(self) -> int:
        """Device bytes this solver holds: the library's resident allocations + result tensors."""
        b = c_size_t()
        check(lib().relu_qp_device_bytes(self._h, byref(b)))
        return b.value + _result_bytes(self.n, self.m, self.batch, self.fp64, self.max_checks)

    def set_tile(self, tile_rows: int):
        check(lib().relu_qp_set_tile(self._h, int(tile_rows)))

    def abort(self):
        check(lib().relu_qp_abort(self._h))

    def set_launch(self, grid: int):
        check(lib().relu_qp_set_launch(self._h, int(grid)))

    def launch(self):
        g, b = c_int(), c_int()
        check(lib().relu_qp_get_launch(self._h, byref(g), byref(b)))
        return g.value, b.value

    def rho_grid(self):
        k = c_int()
        check(lib().relu_qp_get_rho_grid(self._h, None, byref(k)))
        g = np.zeros(k.value)
        check(lib().relu_qp_get_rho_grid(self._h, _ptr(g), byref(k)))
        return g

    def result(self, index: int | None = None) -> dict:
        """Synchronise and copy outputs to the host: instance ``index`` (default: 0 for a single
        instance, all instances as arrays otherwise)."""
        torch.cuda.synchronize(self.device)
        if index is None and self.batch > 1:
            return dict(
                x=self.x.double().cpu().numpy(), y=self.y.double().cpu().numpy(), z=self.z.double().cpu().numpy(),
                iterations=self.iterations.cpu().numpy(), status=self.status.cpu().numpy(),
                rho_index=self.rho_index.cpu().numpy(), rho_hist=self.rho_hist.cpu().numpy(),
                prim_res=self.prim_res.cpu().numpy(), dual_res=self.dual_res.cpu().numpy(),
            )
        b = 0 if index is None else int(index)
        it = int(self.iterations[b].item())
        nck = min(self.max_checks, -(-it // self.settings.check_interval)) if it > 0 else 0
        return dict(
            x=self.x[b].double().cpu().numpy(),
            y=self.y[b].double().cpu().numpy(),
            z=self.z[b].double().cpu().numpy(),
            iterations=it,
            status=int(self.status[b].item()),
            rho_index=int(self.rho_index[b].item()),
            rho_hist=self.rho_hist[b, :nck].cpu().numpy().tolist(),
            prim_res=self.prim_res[b, :nck].cpu().numpy(),
            dual_res=self.dual_res[b, :nck].cpu().numpy(),
        )

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().relu_qp_cleanup(self._h)
            self._h = c_void_p()
        _OPEN.discard(self)

    def __del__(self):
        # during interpreter shutdown the exit hook has already closed every handle; never call
        # into the HIP runtime from a finaliser that late
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
