"""Python handle on the library's serving loop (dc_submit / dc_poll / dc_wait): argument
marshalling only.

Requests carry host arrays; the library copies them at submit time, admits the request when its
device memory fits the context's budget, runs sampling, Chamfer forward and backward for every
frame on the GPU, and returns the per-frame loss and (optionally) the vertex gradient.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


class Server:
    """Submit calibration requests to a context's serving loop and collect their results."""

    def __init__(self, ctx: _lib.Context | None = None, device: int = 0,
                 hbm_budget_bytes: int = 0, max_slots: int = 0):
        self.ctx = ctx or _lib.Context(device, hbm_budget_bytes, max_slots)
        self._live = {}

    def submit(self, verts, faces, observed, n_sim: int, seed: int = 0,
               precision: int = _lib.DC_PREC_BF16_REFINE, reduction: int = _lib.DC_RED_BIDIR_MEAN,
               frame_w=None, want_grad: bool = True) -> int:
        v = np.ascontiguousarray(verts, np.float32)
        f = np.ascontiguousarray(faces, np.int32)
        o = np.ascontiguousarray(observed, np.float32)
        T, V, _ = v.shape
        fw = None if frame_w is None else np.ascontiguousarray(frame_w, np.float32)
        loss = np.zeros(T, np.float64)
        grad = np.zeros((T, V, 3), np.float32) if want_grad else None
        req = _lib.Request(v.ctypes.data, f.ctypes.data, T, V, f.shape[0], n_sim, o.ctypes.data,
                           o.shape[1], seed & (2**64 - 1), precision, reduction,
                           fw.ctypes.data if fw is not None else None)
        res = _lib.Result(loss.ctypes.data, grad.ctypes.data if grad is not None else None,
                          0.0, 0.0, 0.0, 0)
        ticket = ctypes.c_uint64()
        rc = _lib.load().dc_submit(self.ctx.handle, ctypes.byref(req), ctypes.byref(res),
                                   ctypes.byref(ticket))
        _lib._check(rc, "dc_submit")
        # the result struct and its buffers must outlive the request
        self._live[ticket.value] = (res, loss, grad)
        return ticket.value

    @staticmethod
    def footprint(verts, faces, observed, n_sim: int, precision: int = _lib.DC_PREC_BF16_REFINE,
                  want_grad: bool = True) -> int:
        """Device bytes the request holds while admitted (what admission reserves)."""
        T, V = np.shape(verts)[:2]
        req = _lib.Request(None, None, T, V, np.shape(faces)[0], n_sim, None,
                           np.shape(observed)[1], 0, precision, 0, None)
        out = ctypes.c_size_t()
        _lib._check(_lib.load().dc_request_bytes(ctypes.byref(req), int(want_grad),
                                                 ctypes.byref(out)), "dc_request_bytes")
        return out.value

    def poll(self, ticket: int) -> int:
        """DC_PENDING (1) while running; then the final status (0 or a negative code)."""
        return _lib.load().dc_poll(self.ctx.handle, ticket)

    def wait_us(self, ticket: int, timeout_us: int) -> int:
        """dc_wait: sleep in the library until the request finishes or timeout_us passes
        (negative: no limit); DC_PENDING (1) if it is still running, else its final status."""
        return _lib.load().dc_wait(self.ctx.handle, ticket, int(timeout_us))

    def wait(self, ticket: int, timeout: float = 120.0):
        """Block until the request finishes; returns (status, loss, grad, times)."""
        st = self.wait_us(ticket, int(timeout * 1e6))
        if st == _lib.DC_PENDING:
            raise TimeoutError(f"request {ticket} still pending after {timeout} s")
        return self.take(ticket, st)

    def take(self, ticket: int, status: int):
        res, loss, grad = self._live.pop(ticket)
        times = dict(submit=res.t_submit, admit=res.t_admit, done=res.t_done)
        return status, loss, grad, times

    def close(self):
        self.ctx.close()
