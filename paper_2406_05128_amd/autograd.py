"""Differentiable time-varying LP filter as a torch.autograd.Function.

Forward: s = LP_a(e) (paper Sec. 3.2, Eq. 6) by the chunked HIP kernels.  The
forward keeps only the float64 chunk-entry states and chunk transitions
(``saved``) besides its inputs; the backward reruns each chunk from its saved
state to recompute s(t) (no stored output), then runs the single adjoint
recursion of Eq. 12 and emits dL/de = ghat and dL/da_i(t) = -ghat(t) s(t-i)
(Eq. 13), honouring ``needs_input_grad``.
"""
from __future__ import annotations

import threading
from typing import Optional

import torch

from .ops import Plan

_plans: dict = {}
_plans_lock = threading.Lock()


def get_plan(M: int, device: torch.device, chunk: Optional[int] = None) -> Plan:
    key = (device.index, int(M), chunk)
    with _plans_lock:
        p = _plans.get(key)
        if p is None:
            p = Plan(M, device, chunk)
            _plans[key] = p
        return p


class LPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, e: torch.Tensor, a: torch.Tensor, zi: Optional[torch.Tensor], chunk: Optional[int],
                store_s: bool):
        e = e.contiguous()
        a = a.contiguous()
        plan = get_plan(a.shape[-1], e.device, chunk)
        s, _, saved = plan.forward(e, a, zi, save=True)
        ctx.plan = plan
        ctx.store_s = store_s
        if store_s:
            ctx.save_for_backward(e, a, zi, saved, s)
        else:
            ctx.save_for_backward(e, a, zi, saved)
        return s

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        if ctx.store_s:
            e, a, zi, saved, s = ctx.saved_tensors
        else:
            e, a, zi, saved = ctx.saved_tensors
            s = None
        need_e, need_a, need_zi = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        if not (need_e or need_a or need_zi):
            return None, None, None, None, None
        ge, ga, gz = ctx.plan.backward(g.contiguous().float(), a, e, saved, s=s, zi=zi,
                                       need_e=need_e, need_a=need_a, need_zi=bool(need_zi and zi is not None))
        return ge, ga, gz, None, None


def lp(e: torch.Tensor, a: torch.Tensor, zi: Optional[torch.Tensor] = None, chunk: Optional[int] = None,
       store_s: bool = False) -> torch.Tensor:
    """Time-varying all-pole filter s(t) = e(t) - sum_i a_i(t) s(t-i), differentiable in e, a and zi.

    e: float32 [B,T]; a: float32 [B,T,M]; zi: optional float64 [B,M] with zi[b,j-1] = s(-j).
    store_s=True keeps s for the backward instead of recomputing it per chunk.
    """
    return LPFunction.apply(e, a, zi, chunk, store_s)


class LPFramesFunction(torch.autograd.Function):
    """The filter with frame-rate coefficients interpolated in the kernels (Sec. 4.3)."""

    @staticmethod
    def forward(ctx, e: torch.Tensor, A: torch.Tensor, hop: int, zi: Optional[torch.Tensor],
                chunk: Optional[int], store_s: bool):
        e = e.contiguous()
        A = A.contiguous()
        plan = get_plan(A.shape[-1], e.device, chunk)
        s, _, saved = plan.forward_frames(e, A, hop, zi, save=True)
        ctx.plan, ctx.hop, ctx.store_s = plan, hop, store_s
        ctx.save_for_backward(e, A, zi, saved, s if store_s else None)
        return s

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        e, A, zi, saved, s = ctx.saved_tensors
        need_e, need_a, need_zi = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[3]
        if not (need_e or need_a or need_zi):
            return None, None, None, None, None, None
        ge, gA, gz = ctx.plan.backward_frames(g.contiguous().float(), A, ctx.hop, e, saved, s=s, zi=zi,
                                              need_e=need_e, need_a=need_a,
                                              need_zi=bool(need_zi and zi is not None))
        return ge, gA, None, gz, None, None


def lp_frames(e: torch.Tensor, A: torch.Tensor, hop: int, zi: Optional[torch.Tensor] = None,
              chunk: Optional[int] = None, store_s: bool = False) -> torch.Tensor:
    """The filter with frame-rate LP coefficients A [B,F,M] (frame q at sample q*hop,
    F = coef_frames_count(T, hop)) linearly upsampled inside the kernels;
    differentiable in e, A and zi."""
    return LPFramesFunction.apply(e, A, hop, zi, chunk, store_s)


class SFSynthFunction(torch.autograd.Function):
    """y = h * LP_A(gamma (p + C * n)) (Eq. 5 with the output FIR), differentiable in
    p, C, gain, A and h (the noise n is a fixed input)."""

    @staticmethod
    def forward(ctx, p, n, C, gain, A, h, hop: int, chunk: Optional[int]):
        from .sf import SFSynth
        key = (A.shape[-1], hop, C.shape[-1], h.shape[0], p.device, chunk)
        syn = _SF_CACHE.get(key)
        if syn is None:
            syn = _SF_CACHE[key] = SFSynth(A.shape[-1], hop, C.shape[-1], h.shape[0], p.device, chunk)
        y, inner = syn.forward(*(t.contiguous() for t in (p, n, C, gain, A, h)))
        ctx.syn, ctx.inner = syn, inner
        return y

    @staticmethod
    def backward(ctx, gy):
        gp, gC, gg, gA, gh = ctx.syn.backward(gy.contiguous().float(), ctx.inner)
        need = ctx.needs_input_grad
        return (gp if need[0] else None, None, gC if need[2] else None, gg if need[3] else None,
                gA if need[4] else None, gh if need[5] else None, None, None)


_SF_CACHE: dict = {}


def sf_synth(p, n, C, gain, A, h, hop: int, chunk: Optional[int] = None) -> torch.Tensor:
    """Source-filter synthesiser around the LP filter; see SFSynth for the layouts."""
    return SFSynthFunction.apply(p, n, C, gain, A, h, hop, chunk)
