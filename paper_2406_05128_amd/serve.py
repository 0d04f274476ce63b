"""Serving runtime binding: continuous batching of forward-filter jobs (lp_serve_* in include/tvlp.h).

The scheduler, HBM arena, slot states and streams all live in the native
library; this class only stages each job's inputs in pinned host memory and
keeps them alive until the job completes.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import _lib


def _pinned(x, dtype=torch.float32) -> torch.Tensor:
    """x itself if it already is contiguous pinned host memory of `dtype`, else a pinned copy."""
    if isinstance(x, torch.Tensor) and x.device.type == "cpu" and x.dtype == dtype and x.is_contiguous() \
            and x.is_pinned():
        return x
    t = torch.as_tensor(x, dtype=dtype)
    out = torch.empty(t.shape, dtype=dtype, pin_memory=True)
    out.copy_(t)
    return out


class Server:
    """A native continuous-batching server for order-M filter jobs on one GPU."""

    def __init__(self, M: int, budget_bytes: int, max_slots: int = 64, slice_len: int = 0,
                 device: Optional[int] = None):
        lib = _lib.load()
        self.M = int(M)
        dev = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        _lib.check(lib.lp_serve_create(ctypes.byref(h), dev, self.M, int(budget_bytes), int(max_slots),
                                       int(slice_len), 0))
        self._h = h
        self._jobs: Dict[int, Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = {}

    def submit(self, e, a, out: Optional[torch.Tensor] = None) -> int:
        """Queues one job (e [T], a [T, M], host data); returns its ticket.

        Pinned contiguous float32 tensors (also views into a larger pinned
        buffer) are used in place; anything else is first copied to pinned
        memory.  `out` (pinned float32 [T]) receives s; by default a new one.
        """
        e_p = _pinned(e)
        a_p = _pinned(a)
        if e_p.dim() != 1 or a_p.shape != (e_p.shape[0], self.M):
            raise ValueError(f"e must be [T] and a [T, {self.M}]")
        if out is None:
            s_p = torch.empty(e_p.shape, dtype=torch.float32, pin_memory=True)
        else:
            s_p = _pinned(out)
            if s_p is not out or s_p.shape != e_p.shape:
                raise ValueError("out must be a pinned contiguous float32 tensor shaped like e")
        t = ctypes.c_uint64()
        _lib.check(_lib.load().lp_serve_submit(self._h, e_p.shape[0], ctypes.c_void_p(e_p.data_ptr()),
                                               ctypes.c_void_p(a_p.data_ptr()), ctypes.c_void_p(s_p.data_ptr()),
                                               ctypes.byref(t)))
        self._jobs[t.value] = (e_p, a_p, s_p)
        return t.value

    def _finish(self, ticket: int, rc: int, lat: ctypes.c_double):
        if rc == _lib.LP_PENDING:
            return None
        bufs = self._jobs.pop(ticket, None)
        _lib.check(rc)
        return bufs[2].numpy(), lat.value

    def poll(self, ticket: int):
        """(s, latency_ms) once done, None while pending."""
        lat = ctypes.c_double()
        return self._finish(ticket, _lib.load().lp_serve_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(lat)),
                            lat)

    def wait(self, ticket: int, timeout: float = 60.0, device_time: bool = False):
        """(s, latency_ms), or (s, latency_ms, device_ms) with device_time: the job's
        time on the device from its first slice to its last; raises TimeoutError if
        the job is not done in time."""
        lat = ctypes.c_double()
        dev = ctypes.c_double()
        rc = _lib.load().lp_serve_wait(self._h, ctypes.c_uint64(ticket), float(timeout), ctypes.byref(lat),
                                       ctypes.byref(dev))
        if rc == _lib.LP_PENDING:
            raise TimeoutError(f"job {ticket} not done after {timeout} s")
        res = self._finish(ticket, rc, lat)
        return (*res, dev.value) if device_time else res

    def stats(self) -> dict:
        v = [ctypes.c_int64() for _ in range(5)]
        _lib.check(_lib.load().lp_serve_stats(self._h, *[ctypes.byref(x) for x in v]))
        keys = ("iterations", "samples", "jobs_done", "queued", "active")
        return {k: x.value for k, x in zip(keys, v)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().lp_serve_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._jobs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def latency_percentiles(lat_ms) -> dict:
    x = np.asarray(lat_ms, dtype=np.float64)
    return {"p50_ms": float(np.percentile(x, 50)), "p99_ms": float(np.percentile(x, 99)),
            "mean_ms": float(x.mean())}
