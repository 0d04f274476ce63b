"""Torch-facing calls over the C ABI (tensors in, tensors out; marshalling only).

Tensors must live on a ROCm GPU: e, s, g float32 [B,T] (or packed [N]), a float32
[B,T,M] (or [N,M]), zi/zf float64 [B,M].  Work is enqueued on torch's current
stream of the tensors' device.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, name: str, dtype: torch.dtype, dim: int):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (the filter runs only in HIP kernels)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != dim:
        raise ValueError(f"{name} must have {dim} dims, got shape {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """Owns an lp_plan (order M, chunk length, device workspace)."""

    def __init__(self, M: int, device: Optional[torch.device] = None, chunk: Optional[int] = None):
        lib = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = dev
        self.M = int(M)
        h = ctypes.c_void_p()
        _lib.check(lib.lp_plan_create(ctypes.byref(h), dev.index or 0, self.M, 0))
        self._h = h
        if chunk is not None:
            self.set_chunk(chunk)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().lp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def chunk(self) -> int:
        return int(_lib.load().lp_plan_get_chunk(self._h))

    def set_chunk(self, L: int):
        _lib.check(_lib.load().lp_plan_set_chunk(self._h, int(L)))

    def reserve(self, B: int, T: int):
        _lib.check(_lib.load().lp_plan_reserve(self._h, int(B), int(T)))

    def set_timing(self, on: bool = True):
        _lib.check(_lib.load().lp_plan_set_timing(self._h, 1 if on else 0))

    def check_status(self):
        """Synchronise and raise if a scan wave of this plan timed out waiting for a neighbour."""
        _lib.check(_lib.load().lp_plan_status(self._h))

    def reset_timings(self):
        _lib.check(_lib.load().lp_plan_reset_timings(self._h))

    def timings(self) -> dict:
        """{kernel name: (total ms, launches)} accumulated while timing was on (synchronises)."""
        lib = _lib.load()
        n = _lib.check(lib.lp_plan_timings(self._h, None, 0, None, None, 0))
        if n == 0:
            return {}
        NL = 64
        names = ctypes.create_string_buffer(n * NL)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        lib.lp_plan_timings(self._h, ctypes.cast(names, ctypes.c_void_p), NL, ctypes.cast(ms, ctypes.c_void_p),
                            ctypes.cast(cnt, ctypes.c_void_p), n)
        out = {}
        for i in range(n):
            nm = names.raw[i * NL:(i + 1) * NL].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(cnt[i]))
        return out

    def saved_bytes(self, B: int, T: int) -> int:
        return int(_lib.load().lp_saved_bytes(self._h, int(B), int(T)))

    def saved_bytes_varlen(self, B: int, N: int) -> int:
        return int(_lib.load().lp_saved_bytes_varlen(self._h, int(B), int(N)))

    # ------------------------------------------------------------ uniform batches
    def forward(self, e: torch.Tensor, a: torch.Tensor, zi: Optional[torch.Tensor] = None,
                want_zf: bool = False, save: bool = True, out: Optional[torch.Tensor] = None,
                saved_out: Optional[torch.Tensor] = None):
        """s = LP_a(e).  Returns (s, zf or None, saved or None).

        out / saved_out: optional preallocated output and saved-state buffers.
        """
        _need(e, "e", torch.float32, 2)
        _need(a, "a", torch.float32, 3)
        B, T = e.shape
        if a.shape != (B, T, self.M):
            raise ValueError(f"a must have shape {(B, T, self.M)}, got {tuple(a.shape)}")
        if zi is not None:
            _need(zi, "zi", torch.float64, 2)
        s = torch.empty_like(e) if out is None else out
        zf = torch.empty((B, self.M), dtype=torch.float64, device=e.device) if want_zf else None
        if saved_out is not None:
            if saved_out.numel() * saved_out.element_size() < self.saved_bytes(B, T):
                raise ValueError("saved_out is smaller than saved_bytes(B, T)")
            saved = saved_out
        else:
            saved = torch.empty(self.saved_bytes(B, T), dtype=torch.uint8, device=e.device) if save else None
        _lib.check(_lib.load().lp_forward(self._h, B, T, _ptr(e), _ptr(a), _ptr(zi), _ptr(s), _ptr(zf),
                                          _ptr(saved), _stream(e.device)))
        return s, zf, saved

    def backward(self, g: torch.Tensor, a: torch.Tensor, e: Optional[torch.Tensor], saved: torch.Tensor,
                 s: Optional[torch.Tensor] = None, zi: Optional[torch.Tensor] = None,
                 need_e: bool = True, need_a: bool = True, need_zi: bool = False):
        """Returns (grad_e, grad_a, grad_zi) (None where not requested)."""
        _need(g, "g", torch.float32, 2)
        _need(a, "a", torch.float32, 3)
        B, T = g.shape
        ge = torch.empty_like(g) if need_e else None
        ga = torch.empty_like(a) if need_a else None
        gz = torch.empty((B, self.M), dtype=torch.float64, device=g.device) if need_zi else None
        _lib.check(_lib.load().lp_backward(self._h, B, T, _ptr(g), _ptr(a), _ptr(e), _ptr(zi), _ptr(s),
                                           _ptr(saved), _ptr(ge), _ptr(ga), _ptr(gz), _stream(g.device)))
        return ge, ga, gz

    # ------------------------------------------------------------ packed variable-length batches
    def forward_varlen(self, e: torch.Tensor, a: torch.Tensor, offsets: torch.Tensor,
                       zi: Optional[torch.Tensor] = None, want_zf: bool = False, save: bool = True):
        _need(e, "e", torch.float32, 1)
        _need(a, "a", torch.float32, 2)
        _need(offsets, "offsets", torch.int64, 1)
        N = e.shape[0]
        B = offsets.shape[0] - 1
        s = torch.empty_like(e)
        zf = torch.empty((B, self.M), dtype=torch.float64, device=e.device) if want_zf else None
        saved = torch.empty(self.saved_bytes_varlen(B, N), dtype=torch.uint8, device=e.device) if save else None
        _lib.check(_lib.load().lp_forward_varlen(self._h, B, _ptr(offsets), N, _ptr(e), _ptr(a), _ptr(zi),
                                                 _ptr(s), _ptr(zf), _ptr(saved), _stream(e.device)))
        return s, zf, saved

    def backward_varlen(self, g, a, e, offsets, saved, s=None, zi=None, need_e=True, need_a=True,
                        need_zi=False):
        N = g.shape[0]
        B = offsets.shape[0] - 1
        ge = torch.empty_like(g) if need_e else None
        ga = torch.empty_like(a) if need_a else None
        gz = torch.empty((B, self.M), dtype=torch.float64, device=g.device) if need_zi else None
        _lib.check(_lib.load().lp_backward_varlen(self._h, B, _ptr(offsets), N, _ptr(g), _ptr(a), _ptr(e),
                                                  _ptr(zi), _ptr(s), _ptr(saved), _ptr(ge), _ptr(ga), _ptr(gz),
                                                  _stream(g.device)))
        return ge, ga, gz


# ---------------------------------------------------------------- sequential baseline

def forward_plain(e: torch.Tensor, a: torch.Tensor, zi: Optional[torch.Tensor] = None, want_zf: bool = False):
    _need(e, "e", torch.float32, 2)
    _need(a, "a", torch.float32, 3)
    B, T = e.shape
    M = a.shape[2]
    s = torch.empty_like(e)
    zf = torch.empty((B, M), dtype=torch.float64, device=e.device) if want_zf else None
    _lib.check(_lib.load().lp_forward_plain(M, B, T, _ptr(e), _ptr(a), _ptr(zi), _ptr(s), _ptr(zf),
                                            _stream(e.device)))
    return s, zf


def backward_plain(g: torch.Tensor, a: torch.Tensor, s: torch.Tensor, zi: Optional[torch.Tensor] = None,
                   need_a: bool = True, need_zi: bool = False):
    B, T = g.shape
    M = a.shape[2]
    ge = torch.empty_like(g)
    ga = torch.empty_like(a) if need_a else None
    gz = torch.empty((B, M), dtype=torch.float64, device=g.device) if need_zi else None
    _lib.check(_lib.load().lp_backward_plain(M, B, T, _ptr(g), _ptr(a), _ptr(zi), _ptr(s), _ptr(ge), _ptr(ga),
                                             _ptr(gz), _stream(g.device)))
    return ge, ga, gz
