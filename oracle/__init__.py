"""Float64 CPU oracle for the time-varying LP filter (paper Sec. 3.2, Eqs. 6, 12, 13).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product
library never loads it and shares no code with it.

``lp_forward`` / ``lp_backward`` call the plain C routines in
``tvlp_oracle.c`` (built with gcc -O2 -ffp-contract=off -fopenmp, no fast
math).  Inputs are normally the same float32 arrays the GPU path reads; they
are promoted exactly to float64 here (float64 inputs are taken as they are,
for finite-difference checks) and results come back in float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tvlp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the C oracle in place; returns the library path."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_lp_forward.argtypes = [I64, I64, ctypes.c_int, P, P, P, P, P]
        lib.oracle_lp_forward.restype = None
        lib.oracle_lp_backward.argtypes = [I64, I64, ctypes.c_int, P, P, P, P, P, P, P, P]
        lib.oracle_lp_backward.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(x: np.ndarray) -> np.ndarray:
    """Exact promotion of float32 (or pass-through of float64) to contiguous float64."""
    if x.dtype not in (np.float32, np.float64):
        raise TypeError(f"oracle inputs must be float32 or float64, got {x.dtype}")
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x: Optional[np.ndarray]):
    return None if x is None else x.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def lp_forward(e: np.ndarray, a: np.ndarray, zi: Optional[np.ndarray] = None):
    """s = LP_a(e) in float64.  e [B,T], a [B,T,M] (f32 or f64), zi [B,M] = s(-1..-M).

    Returns (s [B,T] f64, zf [B,M] f64 with zf[b, j-1] = s(T-j)).
    """
    e = _f64(e)
    a = _f64(a)
    B, T = e.shape
    M = a.shape[2]
    assert a.shape == (B, T, M)
    zi64 = None if zi is None else np.ascontiguousarray(zi, dtype=np.float64).reshape(B, M)
    s = np.empty((B, T), np.float64)
    zf = np.empty((B, M), np.float64)
    _load().oracle_lp_forward(B, T, M, _ptr(e), _ptr(a), _ptr(zi64), _ptr(s), _ptr(zf))
    return s, zf


def lp_backward(g: np.ndarray, a: np.ndarray, s: np.ndarray, zi: Optional[np.ndarray] = None,
                need_grad_a: bool = True, need_grad_zi: bool = False):
    """Adjoint of lp_forward in float64 (pull form of Eq. 12, then Eq. 13).

    g [B,T] upstream gradient, a [B,T,M] (f32 or f64), s [B,T] f64 from lp_forward.
    Returns (grad_e [B,T], grad_a [B,T,M] or None, grad_zi [B,M] or None), all f64.
    """
    g = _f64(g)
    a = _f64(a)
    B, T = g.shape
    M = a.shape[2]
    s = np.ascontiguousarray(s, dtype=np.float64)
    zi64 = None if zi is None else np.ascontiguousarray(zi, dtype=np.float64).reshape(B, M)
    ge = np.empty((B, T), np.float64)
    ga = np.empty((B, T, M), np.float64) if need_grad_a else None
    gz = np.empty((B, M), np.float64) if need_grad_zi else None
    _load().oracle_lp_backward(B, T, M, _ptr(g), _ptr(a), _ptr(zi64), _ptr(s), _ptr(ge),
                               _ptr(ga), _ptr(gz), None)
    return ge, ga, gz


def lp_forward_ti(e: np.ndarray, a: np.ndarray, zi: Optional[np.ndarray] = None):
    """Time-invariant filter (Sec. 2.2, Eq. 2): one coefficient row a [B,M] used at
    every sample, i.e. Eq. 6 with a_i(t) = a_i.  Returns (s, zf) as lp_forward."""
    B, M = a.shape
    T = e.shape[1]
    return lp_forward(e, np.broadcast_to(_f64(a)[:, None, :], (B, T, M)), zi)


def lp_backward_ti(g: np.ndarray, a: np.ndarray, s: np.ndarray, zi: Optional[np.ndarray] = None,
                   need_grad_zi: bool = False):
    """Adjoint of lp_forward_ti: grad_e and grad_zi as lp_backward; the coefficient
    gradient is dL/da_i = sum_t dL/da_i(t) (the row is shared by every sample;
    Eq. 4).  Returns (grad_e [B,T], grad_a [B,M], grad_zi [B,M] or None)."""
    B, M = a.shape
    T = g.shape[1]
    ge, ga, gz = lp_backward(g, np.broadcast_to(_f64(a)[:, None, :], (B, T, M)), s, zi,
                             need_grad_zi=need_grad_zi)
    return ge, ga.sum(axis=1), gz


def coef_frames_count(T: int, hop: int) -> int:
    """Frame-rate coefficient rows for a length-T signal: frame q sits at sample
    q hop, and the last sample needs a right neighbour, so F = (T - 1) // hop + 2."""
    return (T - 1) // hop + 2


def upsample_frames(A: np.ndarray, T: int, hop: int) -> np.ndarray:
    """Linear upsampling of frame-rate LP coefficients to the sample rate (Sec. 4.3):
    for t = q hop + n (0 <= n < hop), a(t) = (1 - n/hop) A[q] + (n/hop) A[q+1].
    A [B,F,M] with F = coef_frames_count(T, hop).  Returns a [B,T,M] in float64."""
    A = _f64(A)
    B, F, M = A.shape
    assert F == coef_frames_count(T, hop)
    t = np.arange(T)
    q = t // hop
    w = ((t - q * hop) / hop)[None, :, None]
    return (1.0 - w) * A[:, q, :] + w * A[:, q + 1, :]


def upsample_frames_adjoint(ga: np.ndarray, F: int, hop: int) -> np.ndarray:
    """Adjoint of upsample_frames: every sample t = q hop + n hands (1 - n/hop) of
    dL/da(t) to frame q and n/hop of it to frame q + 1.  ga [B,T,M] -> [B,F,M]."""
    ga = np.asarray(ga, dtype=np.float64)
    B, T, M = ga.shape
    gA = np.zeros((B, F, M))
    for q in range(F - 1):
        lo, hi = q * hop, min((q + 1) * hop, T)
        if lo >= hi:
            continue
        w = ((np.arange(lo, hi) - q * hop) / hop)[None, :, None]
        gA[:, q] += ((1.0 - w) * ga[:, lo:hi]).sum(axis=1)
        gA[:, q + 1] += (w * ga[:, lo:hi]).sum(axis=1)
    return gA


def _frame_rows(A: np.ndarray, T: int, hop: int, round_rows: bool) -> np.ndarray:
    """Upsampled rows as the filter reads them: by default rounded once to float32,
    the precision of the per-sample rows (and of a float32 upsampling)."""
    a = upsample_frames(A, T, hop)
    return a.astype(np.float32) if round_rows else a


def lp_forward_frames(e: np.ndarray, A: np.ndarray, hop: int, zi: Optional[np.ndarray] = None,
                      round_rows: bool = True):
    """The filter with frame-rate coefficients A [B,F,M] linearly upsampled to every
    sample (Sec. 4.3), then Eq. 6.  round_rows=False keeps the float64 rows (for
    finite differences).  Returns (s, zf) as lp_forward."""
    return lp_forward(e, _frame_rows(A, e.shape[1], hop, round_rows), zi)


def lp_backward_frames(g: np.ndarray, A: np.ndarray, s: np.ndarray, hop: int,
                       zi: Optional[np.ndarray] = None, need_grad_zi: bool = False, round_rows: bool = True):
    """Adjoint of lp_forward_frames: the per-sample adjoint (Eqs. 12-13) on the
    upsampled rows, then dL/dA by the adjoint of the upsampling (the rounding of
    the rows is taken as the identity).
    Returns (grad_e [B,T], grad_A [B,F,M], grad_zi [B,M] or None)."""
    T = g.shape[1]
    F = A.shape[1]
    ge, ga, gz = lp_backward(g, _frame_rows(A, T, hop, round_rows), s, zi, need_grad_zi=need_grad_zi)
    return ge, upsample_frames_adjoint(ga, F, hop), gz


def framewise_fir(n: np.ndarray, C: np.ndarray, hop: int) -> np.ndarray:
    """Frame-wise FIR filtering (the noise filter C(z) of Eq. 5): each hop-sample
    frame q of the input is convolved with its own taps C[q] and the results
    overlap-add, u(t) = sum_k C[q(t-k)][k] n(t-k) with q(tau) = tau // hop.
    n [B,T], C [B,F,K] (F >= ceil(T / hop)).  Returns u [B,T] in float64."""
    n = _f64(n)
    C = _f64(C)
    B, T = n.shape
    K = C.shape[2]
    u = np.zeros((B, T))
    for q in range(-(-T // hop)):
        lo, hi = q * hop, min((q + 1) * hop, T)
        for b in range(B):
            y = np.convolve(n[b, lo:hi], C[b, q])[: T - lo]
            u[b, lo:lo + len(y)] += y
    return u


def framewise_fir_adjoint(gu: np.ndarray, n: np.ndarray, F: int, K: int, hop: int) -> np.ndarray:
    """dL/dC[q][k] = sum over the samples tau of frame q of dL/du(tau + k) n(tau)."""
    gu = np.asarray(gu, dtype=np.float64)
    n = _f64(n)
    B, T = n.shape
    gC = np.zeros((B, F, K))
    for q in range(-(-T // hop)):
        lo, hi = q * hop, min((q + 1) * hop, T)
        for k in range(K):
            if lo + k >= T:
                break
            m = min(hi, T - k)
            gC[:, q, k] = np.sum(gu[:, lo + k:m + k] * n[:, lo:m], axis=1)
    return gC


def fir(s: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Causal FIR y(t) = sum_k h[k] s(t-k) (the trainable output filter)."""
    s = _f64(s)
    h = _f64(h)
    return np.stack([np.convolve(s[b], h)[: s.shape[1]] for b in range(s.shape[0])])


def fir_adjoint(gy: np.ndarray, s: np.ndarray, h: np.ndarray):
    """Adjoint of fir: dL/ds(t) = sum_k h[k] dL/dy(t+k), dL/dh[k] = sum_b,t dL/dy(t) s(t-k)."""
    gy = np.asarray(gy, dtype=np.float64)
    s = _f64(s)
    h = _f64(h)
    B, T = s.shape
    K = h.shape[0]
    gs = np.stack([np.convolve(gy[b][::-1], h)[:T][::-1] for b in range(B)])
    gh = np.array([np.sum(gy[:, k:] * s[:, :T - k]) if k < T else 0.0 for k in range(K)])
    return gs, gh


def sf_forward(p, n, C, gain, A, h, hop: int, round_rows: bool = True):
    """Source-filter synthesiser of Eq. 5 around the LP filter: the source is the
    pulse train plus frame-wise FIR filtered noise, u = p + C * n; the LP filter
    H takes it through an input gain linearly upsampled from frame values,
    x = gamma u, s = LP_A(x) with frame-rate rows A (Sec. 4.3); the output filter
    is the trainable FIR y = h * s.  gain [B,F], A [B,F,M], C [B,F,K], F =
    coef_frames_count(T, hop).  Returns y and the intermediates (u, gamma, x, s)."""
    T = p.shape[1]
    u = _f64(p) + framewise_fir(n, C, hop)
    gam = upsample_frames(_f64(gain)[..., None], T, hop)[..., 0]
    x = gam * u
    s, _ = lp_forward_frames(x, A, hop, round_rows=round_rows)
    return fir(s, h), (u, gam, x, s)


def sf_backward(gy, n, C, gain, A, h, inter, hop: int, round_rows: bool = True):
    """Adjoint of sf_forward.  Returns (grad_p [B,T], grad_C [B,F,K], grad_gain [B,F],
    grad_A [B,F,M], grad_h [K2])."""
    u, gam, x, s = inter
    F = A.shape[1]
    gs, gh = fir_adjoint(gy, s, h)
    gx, gA, _ = lp_backward_frames(gs, A, s, hop, round_rows=round_rows)
    ggain = upsample_frames_adjoint((gx * u)[..., None], F, hop)[..., 0]
    gu = gam * gx
    gC = framewise_fir_adjoint(gu, n, F, C.shape[2], hop)
    return gu, gC, ggain, gA, gh


def framewise_geometry(T: int, hop: int):
    """Frames of the frame-wise approximation: length W = 4 hop (75 % overlap),
    frame f starting at sample (f - 3) hop, F = ceil(T / hop) + 3 frames, so that
    every sample lies in exactly four frames.  Returns (W, F)."""
    return 4 * hop, -(-T // hop) + 3


def hann_periodic(W: int) -> np.ndarray:
    """w(n) = sin^2(pi n / W), n = 0 .. W-1; at 75 % overlap the shifted copies sum to 2."""
    n = np.arange(W, dtype=np.float64)
    return np.sin(np.pi * n / W) ** 2


def framewise_forward(e: np.ndarray, af: np.ndarray, hop: int):
    """Frame-wise approximation of the time-varying filter (Sec. 3.2, the method of
    the cited frame-wise work): each frame of the excitation is filtered by the
    time-invariant filter of its own coefficient row (Eq. 2, zero initial state),
    and the filtered frames are overlap-added through a Hann window, normalised by
    the window sum (2).  e [B,T], af [B,F,M].  Returns (s [B,T], s_frames [B,F,W])."""
    e = _f64(e)
    af = _f64(af)
    B, T = e.shape
    W, F = framewise_geometry(T, hop)
    assert af.shape[:2] == (B, F)
    M = af.shape[2]
    w = hann_periodic(W)
    ef = np.zeros((B, F, W))
    for f in range(F):
        t0 = (f - 3) * hop
        lo, hi = max(t0, 0), min(t0 + W, T)
        if hi > lo:
            ef[:, f, lo - t0:hi - t0] = e[:, lo:hi]
    sf, _ = lp_forward_ti(ef.reshape(B * F, W), af.reshape(B * F, M))
    sf = sf.reshape(B, F, W)
    s = np.zeros((B, T))
    for f in range(F):
        t0 = (f - 3) * hop
        lo, hi = max(t0, 0), min(t0 + W, T)
        if hi > lo:
            s[:, lo:hi] += 0.5 * w[lo - t0:hi - t0] * sf[:, f, lo - t0:hi - t0]
    return s, sf


def framewise_backward(g: np.ndarray, af: np.ndarray, sf: np.ndarray, hop: int):
    """Adjoint of framewise_forward: dL/ds_f(n) = w(n) g(t0 + n) / 2 inside the
    signal, the time-invariant adjoint per frame (Eqs. 3-4), then dL/de(t) = sum
    over the four frames holding t of dL/de_f.  Returns (grad_e [B,T], grad_af [B,F,M])."""
    g = _f64(g)
    af = _f64(af)
    B, T = g.shape
    W, F = framewise_geometry(T, hop)
    M = af.shape[2]
    w = hann_periodic(W)
    gf = np.zeros((B, F, W))
    for f in range(F):
        t0 = (f - 3) * hop
        lo, hi = max(t0, 0), min(t0 + W, T)
        if hi > lo:
            gf[:, f, lo - t0:hi - t0] = 0.5 * w[lo - t0:hi - t0] * g[:, lo:hi]
    gef, gaf, _ = lp_backward_ti(gf.reshape(B * F, W), af.reshape(B * F, M), sf.reshape(B * F, W))
    gef = gef.reshape(B, F, W)
    ge = np.zeros((B, T))
    for f in range(F):
        t0 = (f - 3) * hop
        lo, hi = max(t0, 0), min(t0 + W, T)
        if hi > lo:
            ge[:, lo:hi] += gef[:, f, lo - t0:hi - t0]
    return ge, gaf.reshape(B, F, M)
