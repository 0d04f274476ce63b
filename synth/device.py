"""Device-side construction of large coefficient tracks (torch, float64 -> float32).

Same recipe as `inputs.make_coeffs` (frame-rate reflection coefficients drawn on
the host, linear interpolation to every sample, step-up recursion, optional
bandwidth expansion), evaluated with torch on a GPU so that workloads of
hundreds of millions of samples can be built in seconds.  Like the rest of
`synth`, it holds none of the filter's own arithmetic.
"""
from __future__ import annotations

import numpy as np

from .inputs import HOP, draw_reflection_frames, make_excitation, make_upstream_grad


def _step_up(k):
    """Step-up recursion on a torch tensor k[..., M] (float64), coefficient-major inside."""
    import torch
    M = k.shape[-1]
    kt = k.movedim(-1, 0).contiguous()
    at = torch.zeros_like(kt)
    for m in range(1, M + 1):
        km = kt[m - 1]
        if m > 1:
            prev = at[: m - 1].clone()
            at[: m - 1] = prev + km * prev.flip(0)
        at[m - 1] = km
    return at.movedim(0, -1).contiguous()


def coeffs_from_frames(kf: np.ndarray, T: int, gamma: float, device, seqs_per_pass: int = 16):
    """a[B, T, M] float32 on `device` from frame-rate reflection coefficients kf[B, F, M]."""
    import torch
    B, F, M = kf.shape
    out = torch.empty((B, T, M), dtype=torch.float32, device=device)
    t = torch.arange(T, device=device)
    f = t // HOP
    alpha = ((t - f * HOP).to(torch.float64) / HOP)[None, :, None]
    scale = torch.tensor([gamma ** i for i in range(1, M + 1)], dtype=torch.float64, device=device)
    for b0 in range(0, B, seqs_per_pass):
        b1 = min(B, b0 + seqs_per_pass)
        kfb = torch.from_numpy(np.ascontiguousarray(kf[b0:b1])).to(device)
        k = (1.0 - alpha) * kfb[:, f, :] + alpha * kfb[:, f + 1, :]
        a = _step_up(k)
        if gamma != 1.0:
            a = a * scale
        out[b0:b1] = a.to(torch.float32)
        del kfb, k, a
    return out


def stress_inputs(B: int, T: int, M: int, kappa: float, gamma: float, seed: int, device,
                  family: str = "randomwalk"):
    """(e, a, g) on `device` for the long high-resonance workload (frames and noise drawn on the host)."""
    import torch
    rng = np.random.default_rng(seed)
    kf = draw_reflection_frames(rng, B, T, M, kappa, family)
    a = coeffs_from_frames(kf, T, gamma, device)
    e = torch.from_numpy(make_excitation(rng, B, T)).to(device)
    g = torch.from_numpy(make_upstream_grad(rng, B, T)).to(device)
    return e, a, g
