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
