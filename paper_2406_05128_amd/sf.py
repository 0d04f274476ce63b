"""Source-filter synthesiser around the LP filter (Eq. 5): S = (G + N C) H, then the
trainable output FIR.

Every step runs in the library's HIP kernels: the source (frame-wise FIR noise
filter plus the pulse train, times the linearly upsampled input gain), the LP
filter with frame-rate coefficients (lp_forward_frames / lp_backward_frames)
and the output FIR, with their adjoints.  Frames: frame q at sample q*hop,
F = coef_frames_count(T, hop) rows for the gain, the noise-filter taps and the
LP coefficients.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _lib
from .ops import Plan, _need, _ptr, _stream, coef_frames_count


class SFSynth:
    """Forward / adjoint of y = h * LP_A(gamma (p + C * n)) for batches [B,T].

    M: LP order; hop: samples per frame; K: noise-filter taps per frame; K2:
    output-FIR taps.  `chunk` is the LP plan's chunk length (None: default).
    """

    def __init__(self, M: int, hop: int, K: int, K2: int, device, chunk: Optional[int] = None):
        self.M, self.hop, self.K, self.K2 = M, hop, K, K2
        self.device = torch.device(device)
        self.plan = Plan(M, self.device, chunk)

    def forward(self, p, n, C, gain, A, h):
        """p, n [B,T]; C [B,F,K]; gain [B,F]; A [B,F,M]; h [K2] -> (y [B,T], ctx)."""
        for t, name, dim in ((p, "p", 2), (n, "n", 2), (C, "C", 3), (gain, "gain", 2), (A, "A", 3), (h, "h", 1)):
            _need(t, name, torch.float32, dim)
        B, T = p.shape
        F = coef_frames_count(T, self.hop)
        if C.shape != (B, F, self.K) or gain.shape != (B, F) or h.shape != (self.K2,):
            raise ValueError("C must be [B,F,K], gain [B,F], h [K2]")
        lib, st = _lib.load(), _stream(p.device)
        u = torch.empty_like(p)
        x = torch.empty_like(p)
        _lib.check_sf(lib.lp_sf_source(B, T, self.hop, self.K, _ptr(p), _ptr(n), _ptr(C), _ptr(gain), _ptr(u),
                                       _ptr(x), st))
        s, _, saved = self.plan.forward_frames(x, A, self.hop)
        y = torch.empty_like(p)
        _lib.check_sf(lib.lp_fir(B, T, self.K2, _ptr(s), _ptr(h), _ptr(y), st))
        return y, (n, C, gain, A, h, u, x, s, saved)

    def backward(self, gy, ctx):
        """gy = dL/dy [B,T] -> (grad_p [B,T], grad_C [B,F,K], grad_gain [B,F], grad_A [B,F,M], grad_h [K2])."""
        _need(gy, "gy", torch.float32, 2)
        n, C, gain, A, h, u, x, s, saved = ctx
        B, T = gy.shape
        lib, st = _lib.load(), _stream(gy.device)
        gs = torch.empty_like(gy)
        gh = torch.empty_like(h)
        work = torch.empty(max(1, lib.lp_fir_adjoint_work_bytes(B, T, self.K2)), dtype=torch.uint8,
                           device=gy.device)
        _lib.check_sf(lib.lp_fir_adjoint(B, T, self.K2, _ptr(gy), _ptr(s), _ptr(h), _ptr(gs), _ptr(gh),
                                         _ptr(work), st))
        gx, gA, _ = self.plan.backward_frames(gs, A, self.hop, x, saved, s=s)
        gp = torch.empty_like(gy)
        gC = torch.empty_like(C)
        ggain = torch.empty_like(gain)
        _lib.check_sf(lib.lp_sf_source_adjoint(B, T, self.hop, self.K, _ptr(gx), _ptr(u), _ptr(n), _ptr(gain),
                                               _ptr(gp), _ptr(gC), _ptr(ggain), st))
        return gp, gC, ggain, gA, gh
