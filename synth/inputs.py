"""Seeded generators for speech-shaped LP filter inputs.

Recipe (the paper's vocoder setting, Sec. 4.1-4.3: 24 kHz audio, 2 s training
segments, batch 64, 10 ms = 240-sample analysis hop, reflection-coefficient
parameterisation of the LP filter, LPCs upsampled to the sample rate):

* Reflection coefficients k_j (j = 1..M) are drawn once per 240-sample frame,
  frame f sitting at sample 240 f, F = floor((T-1)/240) + 2 frames so that the
  last sample has a right neighbour.
* k is linearly interpolated to every sample, then converted to direct-form LP
  coefficients a_i(t) with the step-up (Levinson) recursion, in float64.
  With |k_j| < 1 every frozen polynomial z^M + a_1 z^(M-1) + ... + a_M has all
  roots inside the unit circle.
* An optional bandwidth expansion a_i <- gamma^i a_i pulls every frozen root
  inside radius gamma; gamma = 0.98 is the "gated" input mode used for the
  1e-4 accuracy gate, gamma = 1 the literal mode.
* Everything is built in float64 and cast to float32 once; both the oracle and
  the GPU path read those float32 arrays.

Nothing here evaluates the filter itself.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

HOP = 240

__all__ = [
    "HOP", "reflection_to_lpc", "interp_frames", "draw_reflection_frames",
    "make_coeffs", "make_excitation", "make_upstream_grad", "pulse_train",
    "poisson_requests", "max_pole_radius", "Workload", "workload",
    "WORKLOADS",
]


def reflection_to_lpc(k: np.ndarray) -> np.ndarray:
    """Step-up recursion: reflection coefficients k[..., M] -> a[..., M].

    Convention A(z) = 1 + sum_i a_i z^-i:
      a^(m)_m = k_m,   a^(m)_i = a^(m-1)_i + k_m a^(m-1)_(m-i)  (i < m).
    Computed in float64 over all leading axes at once.
    """
    k = np.asarray(k, dtype=np.float64)
    M = k.shape[-1]
    # coefficient-major copy: every update below streams contiguous rows
    kt = np.ascontiguousarray(np.moveaxis(k, -1, 0))
    at = np.zeros_like(kt)
    for m in range(1, M + 1):
        km = kt[m - 1]
        if m > 1:
            prev = at[: m - 1].copy()
            at[: m - 1] = prev + km * prev[::-1]
        at[m - 1] = km
    return np.ascontiguousarray(np.moveaxis(at, 0, -1))


def interp_frames(frames: np.ndarray, T: int, hop: int = HOP) -> np.ndarray:
    """Linear interpolation of per-frame values [B, F, M] to per-sample [B, T, M]."""
    t = np.arange(T)
    f = t // hop
    alpha = ((t - f * hop) / hop)[None, :, None]
    return (1.0 - alpha) * frames[:, f, :] + alpha * frames[:, f + 1, :]


def n_frames(T: int, hop: int = HOP) -> int:
    return (T - 1) // hop + 2


def draw_reflection_frames(rng: np.random.Generator, B: int, T: int, M: int,
                           kappa: float, family: str = "iid",
                           walk_sigma: float = 0.01) -> np.ndarray:
    """Frame-rate reflection coefficients [B, F, M] for one of three families.

    iid        : every frame k ~ U(-kappa, kappa) independently.
    randomwalk : k_0 ~ U(-kappa, kappa), k_f = clip(k_(f-1) + N(0, sigma^2), +-kappa).
    ti         : one draw per sequence, held constant (time-invariant filter).
    """
    F = n_frames(T)
    if family == "iid":
        return rng.uniform(-kappa, kappa, size=(B, F, M))
    if family == "randomwalk":
        k = np.empty((B, F, M))
        k[:, 0] = rng.uniform(-kappa, kappa, size=(B, M))
        steps = rng.normal(0.0, walk_sigma, size=(B, F - 1, M))
        for f in range(1, F):
            k[:, f] = np.clip(k[:, f - 1] + steps[:, f - 1], -kappa, kappa)
        return k
    if family == "ti":
        k0 = rng.uniform(-kappa, kappa, size=(B, 1, M))
        return np.repeat(k0, F, axis=1)
    raise ValueError(f"unknown coefficient family {family!r}")


def make_coeffs(rng: np.random.Generator, B: int, T: int, M: int, kappa: float,
                gamma: float = 1.0, family: str = "iid",
                dtype=np.float32) -> np.ndarray:
    """Per-sample LP coefficients a[B, T, M] (row t multiplies s(t-1..t-M) to make s(t))."""
    kf = draw_reflection_frames(rng, B, T, M, kappa, family)
    a = np.empty((B, T, M), dtype=dtype)
    # one sequence at a time keeps the float64 temporaries small
    for b in range(B):
        k = interp_frames(kf[b:b + 1], T)[0]
        ab = reflection_to_lpc(k)
        if gamma != 1.0:
            ab *= gamma ** np.arange(1, M + 1, dtype=np.float64)
        a[b] = ab.astype(dtype)
    return a


def make_excitation(rng: np.random.Generator, B: int, T: int, dtype=np.float32) -> np.ndarray:
    """White Gaussian excitation e(t) ~ N(0, 1), shape [B, T]."""
    return rng.standard_normal((B, T)).astype(dtype)


def make_upstream_grad(rng: np.random.Generator, B: int, T: int, dtype=np.float32) -> np.ndarray:
    """Upstream gradient dL/ds(t) ~ N(0, 1), shape [B, T]."""
    return rng.standard_normal((B, T)).astype(dtype)


def pulse_train(rng: np.random.Generator, B: int, T: int, pmin: int = 100, pmax: int = 400,
                dtype=np.float32) -> np.ndarray:
    """Glottal-like impulse trains, one per item.

    Integer period P ~ U{pmin..pmax}, phase ~ U{0..P-1}, amplitude A ~ U(0.1, 1);
    pulses of height A at t = phase + n P.
    """
    x = np.zeros((B, T), dtype=dtype)
    for b in range(B):
        P = int(rng.integers(pmin, pmax + 1))
        phase = int(rng.integers(0, P))
        amp = float(rng.uniform(0.1, 1.0))
        x[b, phase::P] = amp
    return x


def poisson_requests(rng: np.random.Generator, n: int, rate_hz: float,
                     tmin: int, tmax: int) -> tuple[np.ndarray, np.ndarray]:
    """Open-loop Poisson arrivals: (arrival times in seconds, lengths in samples)."""
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    arrivals = np.cumsum(gaps)
    lengths = rng.integers(tmin, tmax + 1, size=n)
    return arrivals, lengths


def max_pole_radius(a: np.ndarray, sample_rows: Optional[np.ndarray] = None) -> float:
    """Largest root modulus of z^M + a_1 z^(M-1) + ... + a_M over the given rows of a[..., M]."""
    rows = np.asarray(a, dtype=np.float64).reshape(-1, a.shape[-1])
    if sample_rows is not None:
        rows = rows[sample_rows]
    r = 0.0
    for row in rows:
        roots = np.roots(np.concatenate([[1.0], row]))
        if roots.size:
            r = max(r, float(np.abs(roots).max()))
    return r


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named synthetic workload: shapes plus the coefficient recipe."""
    name: str
    B: int
    T: int
    M: int
    kappa: float
    family: str = "iid"
    seed: int = 0

    @property
    def samples(self) -> int:
        return self.B * self.T


WORKLOADS = {
    # small parity case: 4 x 16000 samples, order 16, |k| < 0.9
    "small_m16": Workload("small_m16", 4, 16000, 16, 0.9, "iid", 1000),
    # training shape: batch 64 of 2 s at 24 kHz, order 22, |k| < 0.95
    "train_b64_t48000_m22": Workload("train_b64_t48000_m22", 64, 48000, 22, 0.95, "iid", 1001),
    # harmonic-plus-noise pair: batch 32 of 4 s, order 22 for both filters
    "hpn_pair_b32_t96000_m22": Workload("hpn_pair_b32_t96000_m22", 32, 96000, 22, 0.95, "iid", 1002),
    # long high-resonance stress case: 512 x 10 s, order 32, bounded random-walk reflections
    "stress_b512_t240000_m32": Workload("stress_b512_t240000_m32", 512, 240000, 32, 0.995,
                                         "randomwalk", 1004),
}


def workload(name: str, gamma: float = 1.0, B: Optional[int] = None, T: Optional[int] = None,
             with_grad: bool = True, seed_offset: int = 0):
    """Build (e, a, g) float32 arrays for a named workload (optionally resized)."""
    w = WORKLOADS[name]
    B = w.B if B is None else B
    T = w.T if T is None else T
    rng = np.random.default_rng(w.seed + seed_offset)
    a = make_coeffs(rng, B, T, w.M, w.kappa, gamma, w.family)
    e = make_excitation(rng, B, T)
    g = make_upstream_grad(rng, B, T) if with_grad else None
    return e, a, g
