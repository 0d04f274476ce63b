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


def _tag_saved(saved: Optional[torch.Tensor], plan: "Plan", B: int, T: int):
    """Record on a saved-state buffer the plan, chunk length and shape it was written
    with: its layout (chunk states and transitions) depends on all of them."""
    if saved is not None:
        saved._tvlp_layout = (id(plan), plan.chunk, int(B), int(T))


def _check_saved(saved: torch.Tensor, plan: "Plan", B: int, T: int, nbytes: int):
    if not isinstance(saved, torch.Tensor):
        raise TypeError("saved must be the tensor returned by the forward")
    if saved.device.type != "cuda" or (saved.device.index or 0) != (plan.device.index or 0):
        raise ValueError("saved lives on another device than the plan")
    if saved.numel() * saved.element_size() < nbytes:
        raise ValueError(f"saved holds {saved.numel() * saved.element_size()} bytes, the backward of "
                         f"B={B}, T={T} at chunk {plan.chunk} needs {nbytes}")
    tag = getattr(saved, "_tvlp_layout", None)
    if tag is not None and tag != (id(plan), plan.chunk, int(B), int(T)):
        raise ValueError(f"saved was written by a forward with (plan, chunk, B, T) = {tag[1:]} on "
                         f"{'this' if tag[0] == id(plan) else 'another'} plan; this backward runs "
                         f"chunk {plan.chunk}, B={B}, T={T} (the saved layout depends on the chunk length)")


def _check_flags(t: Optional[torch.Tensor], B: int):
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.int32 \
            or t.dim() != 1 or t.shape[0] < B or not t.is_contiguous():
        raise ValueError(f"nonfinite must be a contiguous int32 GPU tensor of at least {B} elements")


def _check_same(t: Optional[torch.Tensor], name: str, shape):
    if t is None:
        return
    _need(t, name, torch.float32, len(shape))
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Plan:
    """Owns an lp_plan (order M, chunk length, device workspace)."""

    def __init__(self, M: int, device: Optional[torch.device] = None, chunk: Optional[int] = None,
                 chained: bool = False, high_radius: bool = False):
        """chained: LP_FLAG_CHAINED_CARRY (carry chunk by chunk, for strongly resonant inputs;
        fixes the carry mode, which the autotuner otherwise picks).
        high_radius: LP_FLAG_HIGH_RADIUS (poles near the unit circle: the chained carry over
        chunks long enough for its accuracy; the autotuner keeps to such lengths)."""
        lib = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = dev
        self.M = int(M)
        self.high_radius = bool(high_radius)
        self._carry_fixed = bool(chained) or self.high_radius
        h = ctypes.c_void_p()
        _lib.check(lib.lp_plan_create(ctypes.byref(h), dev.index or 0, self.M,
                                      (_lib.LP_FLAG_CHAINED_CARRY if chained else 0)
                                      | (_lib.LP_FLAG_HIGH_RADIUS if high_radius else 0)))
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

    @property
    def chained(self) -> bool:
        """Whether the plan carries chunk by chunk (else through group maps)."""
        return _lib.load().lp_plan_get_carry(self._h) == 1

    def set_carry(self, chained: bool):
        """Fix the carry mode (lp_plan_set_carry); the autotuner then keeps it."""
        _lib.check(_lib.load().lp_plan_set_carry(self._h, 1 if chained else 0))
        self._carry_fixed = True

    def reserve(self, B: int, T: int):
        _lib.check(_lib.load().lp_plan_reserve(self._h, int(B), int(T)))

    def autotune(self, B: int, T: int, reps: int = 3, cache: bool = True) -> dict:
        """Pick the fastest chunk length (and, unless fixed, carry mode) for a B x T
        forward + adjoint step (lp_plan_autotune).

        Results are cached per (device name, M, B, T, carry constraint, library build) in a JSON file
        ($TVLP_AUTOTUNE_CACHE, default ~/.cache/tvlp/autotune.json); a cached
        entry is applied without measuring.  Returns {"chunk", "chained", "ms", "cached"}.
        """
        from . import autotune as _at
        constraint = ("high-radius" if self.high_radius
                      else (("chained" if self.chained else "grouped") if self._carry_fixed else "free"))
        key = _at.cache_key(torch.cuda.get_device_name(self.device), self.M, B, T, constraint, _lib.build_id())
        if cache:
            hit = _at.lookup(key)
            if hit is not None:
                self.set_chunk(hit["chunk"])
                if not self._carry_fixed:
                    # apply the cached mode and leave the choice free for later tuning
                    _lib.check(_lib.load().lp_plan_set_carry(self._h, 1 if hit["chained"] else 0))
                    _lib.check(_lib.load().lp_plan_set_carry(self._h, -1))
                return {**hit, "chained": self.chained, "cached": True}
        L = ctypes.c_int()
        ms = ctypes.c_double()
        _lib.check(_lib.load().lp_plan_autotune(self._h, int(B), int(T), int(reps), ctypes.byref(L),
                                                ctypes.byref(ms)))
        res = {"chunk": int(L.value), "chained": self.chained, "ms": float(ms.value)}
        if cache:
            _at.store(key, res)
        return {**res, "cached": False}

    def set_timing(self, on: bool = True):
        _lib.check(_lib.load().lp_plan_set_timing(self._h, 1 if on else 0))

    def check_status(self):
        """Synchronise; raise if a segment table held more samples than its total_bound (LP_EINVAL,
        clears the flag) or the device reports an error (LP_EDEVICE)."""
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
                saved_out: Optional[torch.Tensor] = None, nonfinite: Optional[torch.Tensor] = None):
        """s = LP_a(e).  Returns (s, zf or None, saved or None).

        out / saved_out: optional preallocated output and saved-state buffers.
        nonfinite: optional int32 [B] device tensor; the call sets element b to 1
        when some output of sequence b is Inf or NaN, else 0.
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
        _check_flags(nonfinite, B)
        _lib.check(_lib.load().lp_forward(self._h, B, T, _ptr(e), _ptr(a), _ptr(zi), _ptr(s), _ptr(zf),
                                          _ptr(saved), _ptr(nonfinite), _stream(e.device)))
        _tag_saved(saved, self, B, T)
        return s, zf, saved

    def forward_ti(self, e: torch.Tensor, a: torch.Tensor, zi: Optional[torch.Tensor] = None,
                   want_zf: bool = False, save: bool = True):
        """Time-invariant coefficients: e [B,T], a [B,M] -> (s, zf or None, saved or None)."""
        _need(e, "e", torch.float32, 2)
        _need(a, "a", torch.float32, 2)
        B, T = e.shape
        if a.shape != (B, self.M):
            raise ValueError(f"a must have shape {(B, self.M)}, got {tuple(a.shape)}")
        if zi is not None:
            _need(zi, "zi", torch.float64, 2)
        s = torch.empty_like(e)
        zf = torch.empty((B, self.M), dtype=torch.float64, device=e.device) if want_zf else None
        saved = torch.empty(self.saved_bytes(B, T), dtype=torch.uint8, device=e.device) if save else None
        _lib.check(_lib.load().lp_forward_ti(self._h, B, T, _ptr(e), _ptr(a), _ptr(zi), _ptr(s), _ptr(zf),
                                             _ptr(saved), _stream(e.device)))
        _tag_saved(saved, self, B, T)
        return s, zf, saved

    def backward_ti(self, g: torch.Tensor, a: torch.Tensor, e: Optional[torch.Tensor], saved: torch.Tensor,
                    s: Optional[torch.Tensor] = None, zi: Optional[torch.Tensor] = None,
                    need_e: bool = True, need_a: bool = True, need_zi: bool = False):
        """Time-invariant coefficients: returns (grad_e [B,T], grad_a [B,M], grad_zi [B,M])."""
        _need(g, "g", torch.float32, 2)
        _need(a, "a", torch.float32, 2)
        B, T = g.shape
        if a.shape != (B, self.M):
            raise ValueError(f"a must have shape {(B, self.M)}, got {tuple(a.shape)}")
        _check_same(e, "e", (B, T))
        _check_same(s, "s", (B, T))
        if zi is not None:
            _need(zi, "zi", torch.float64, 2)
        _check_saved(saved, self, B, T, self.saved_bytes(B, T))
        ge = torch.empty_like(g) if need_e else None
        ga = torch.empty_like(a) if need_a else None
        gz = torch.empty((B, self.M), dtype=torch.float64, device=g.device) if need_zi else None
        _lib.check(_lib.load().lp_backward_ti(self._h, B, T, _ptr(g), _ptr(a), _ptr(e), _ptr(zi), _ptr(s),
                                              _ptr(saved), _ptr(ge), _ptr(ga), _ptr(gz), _stream(g.device)))
        return ge, ga, gz

    def forward_frames(self, e: torch.Tensor, A: torch.Tensor, hop: int, zi: Optional[torch.Tensor] = None,
                       want_zf: bool = False, save: bool = True):
        """Frame-rate coefficients: e [B,T], A [B,F,M] (frame q at sample q*hop, F =
        coef_frames_count(T, hop)), interpolated per sample inside the kernels
        -> (s, zf or None, saved or None)."""
        _need(e, "e", torch.float32, 2)
        _need(A, "A", torch.float32, 3)
        B, T = e.shape
        F = coef_frames_count(T, hop)
        if A.shape != (B, F, self.M):
            raise ValueError(f"A must have shape {(B, F, self.M)}, got {tuple(A.shape)}")
        if zi is not None:
            _need(zi, "zi", torch.float64, 2)
        s = torch.empty_like(e)
        zf = torch.empty((B, self.M), dtype=torch.float64, device=e.device) if want_zf else None
        saved = torch.empty(self.saved_bytes(B, T), dtype=torch.uint8, device=e.device) if save else None
        _lib.check(_lib.load().lp_forward_frames(self._h, B, T, int(hop), _ptr(e), _ptr(A), _ptr(zi), _ptr(s),
                                                 _ptr(zf), _ptr(saved), _stream(e.device)))
        _tag_saved(saved, self, B, T)
        return s, zf, saved

    def backward_frames(self, g: torch.Tensor, A: torch.Tensor, hop: int, e: Optional[torch.Tensor],
                        saved: torch.Tensor, s: Optional[torch.Tensor] = None, zi: Optional[torch.Tensor] = None,
                        need_e: bool = True, need_a: bool = True, need_zi: bool = False):
        """Frame-rate coefficients: returns (grad_e [B,T], grad_A [B,F,M], grad_zi [B,M])."""
        _need(g, "g", torch.float32, 2)
        _need(A, "A", torch.float32, 3)
        B, T = g.shape
        F = coef_frames_count(T, hop)
        if A.shape != (B, F, self.M):
            raise ValueError(f"A must have shape {(B, F, self.M)}, got {tuple(A.shape)}")
        _check_same(e, "e", (B, T))
        _check_same(s, "s", (B, T))
        if zi is not None:
            _need(zi, "zi", torch.float64, 2)
        _check_saved(saved, self, B, T, self.saved_bytes(B, T))
        ge = torch.empty_like(g) if need_e else None
        gA = torch.empty_like(A) if need_a else None
        gz = torch.empty((B, self.M), dtype=torch.float64, device=g.device) if need_zi else None
        _lib.check(_lib.load().lp_backward_frames(self._h, B, T, int(hop), _ptr(g), _ptr(A), _ptr(e), _ptr(zi),
                                                  _ptr(s), _ptr(saved), _ptr(ge), _ptr(gA), _ptr(gz),
                                                  _stream(g.device)))
        return ge, gA, gz

    def backward(self, g: torch.Tensor, a: torch.Tensor, e: Optional[torch.Tensor], saved: torch.Tensor,
                 s: Optional[torch.Tensor] = None, zi: Optional[torch.Tensor] = None,
                 need_e: bool = True, need_a: bool = True, need_zi: bool = False,
                 nonfinite: Optional[torch.Tensor] = None):
        """Returns (grad_e, grad_a, grad_zi) (None where not requested).  nonfinite:
        optional int32 [B] device tensor, set to 1 where a sequence's gradients hold
        Inf or NaN, else 0."""
        _need(g, "g", torch.float32, 2)
        _need(a, "a", torch.float32, 3)
        B, T = g.shape
        if a.shape != (B, T, self.M):
            raise ValueError(f"a must have shape {(B, T, self.M)}, got {tuple(a.shape)}")
        _check_same(e, "e", (B, T))
        _check_same(s, "s", (B, T))
        if zi is not None:
            _need(zi, "zi", torch.float64, 2)
        _check_saved(saved, self, B, T, self.saved_bytes(B, T))
        ge = torch.empty_like(g) if need_e else None
        ga = torch.empty_like(a) if need_a else None
        gz = torch.empty((B, self.M), dtype=torch.float64, device=g.device) if need_zi else None
        _check_flags(nonfinite, B)
        _lib.check(_lib.load().lp_backward(self._h, B, T, _ptr(g), _ptr(a), _ptr(e), _ptr(zi), _ptr(s),
                                           _ptr(saved), _ptr(ge), _ptr(ga), _ptr(gz), _ptr(nonfinite),
                                           _stream(g.device)))
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
        _tag_saved(saved, self, B, N)
        return s, zf, saved

    def backward_varlen(self, g, a, e, offsets, saved, s=None, zi=None, need_e=True, need_a=True,
                        need_zi=False):
        _need(g, "g", torch.float32, 1)
        _need(a, "a", torch.float32, 2)
        _need(offsets, "offsets", torch.int64, 1)
        N = g.shape[0]
        B = offsets.shape[0] - 1
        if a.shape != (N, self.M):
            raise ValueError(f"a must have shape {(N, self.M)}, got {tuple(a.shape)}")
        _check_same(e, "e", (N,))
        _check_same(s, "s", (N,))
        _check_saved(saved, self, B, N, self.saved_bytes_varlen(B, N))
        ge = torch.empty_like(g) if need_e else None
        ga = torch.empty_like(a) if need_a else None
        gz = torch.empty((B, self.M), dtype=torch.float64, device=g.device) if need_zi else None
        _lib.check(_lib.load().lp_backward_varlen(self._h, B, _ptr(offsets), N, _ptr(g), _ptr(a), _ptr(e),
                                                  _ptr(zi), _ptr(s), _ptr(saved), _ptr(ge), _ptr(ga), _ptr(gz),
                                                  _stream(g.device)))
        return ge, ga, gz

    # ------------------------------------------------------------ segment tables (serving)
    def forward_segments(self, e: torch.Tensor, a: torch.Tensor, starts: torch.Tensor, lens: torch.Tensor,
                         state: Optional[torch.Tensor] = None, s: Optional[torch.Tensor] = None,
                         total_bound: int = 0):
        """Sequence b = samples [starts[b], starts[b] + lens[b]) of e [N], a [N,M]; non-overlapping.

        `state` float64 [B,M] is read as the initial state and overwritten with the
        final state of every sequence with lens[b] > 0 (in place).  Returns s [N]
        (only the covered samples are written).
        """
        _need(e, "e", torch.float32, 1)
        _need(a, "a", torch.float32, 2)
        _need(starts, "starts", torch.int64, 1)
        _need(lens, "lens", torch.int64, 1)
        N = e.shape[0]
        B = starts.shape[0]
        if lens.shape[0] != B:
            raise ValueError("starts and lens must have the same length")
        if state is not None:
            _need(state, "state", torch.float64, 2)
            if state.shape != (B, self.M):
                raise ValueError(f"state must have shape {(B, self.M)}")
        if s is None:
            s = torch.empty_like(e)
        else:
            _need(s, "s", torch.float32, 1)
        _lib.check(_lib.load().lp_forward_segments(self._h, B, _ptr(starts), _ptr(lens), N, int(total_bound),
                                                   _ptr(e), _ptr(a), _ptr(state), _ptr(s), _ptr(state),
                                                   _stream(e.device)))
        return s

    # ------------------------------------------------------------ filter pair (Eq. 1)
    def saved_bytes_pair(self, B: int, T: int) -> int:
        return int(_lib.load().lp_saved_bytes_pair(self._h, int(B), int(T)))

    def forward_pair(self, e2: torch.Tensor, a2: torch.Tensor, y: Optional[torch.Tensor] = None,
                     s2: Optional[torch.Tensor] = None, saved: Optional[torch.Tensor] = None):
        """Two filters per item, stacked: e2 [2,B,T], a2 [2,B,T,M] -> (y = s2[0] + s2[1], s2, saved)."""
        _need(e2, "e2", torch.float32, 3)
        _need(a2, "a2", torch.float32, 4)
        _, B, T = e2.shape
        if a2.shape != (2, B, T, self.M):
            raise ValueError(f"a2 must have shape {(2, B, T, self.M)}")
        if y is None:
            y = torch.empty((B, T), dtype=torch.float32, device=e2.device)
        else:
            _need(y, "y", torch.float32, 2)
            if y.shape != (B, T):
                raise ValueError(f"y must have shape {(B, T)}")
        if s2 is None:
            s2 = torch.empty_like(e2)
        else:
            _need(s2, "s2", torch.float32, 3)
            if s2.shape != e2.shape:
                raise ValueError(f"s2 must have shape {tuple(e2.shape)}")
        if saved is None:
            saved = torch.empty(self.saved_bytes_pair(B, T), dtype=torch.uint8, device=e2.device)
        _lib.check(_lib.load().lp_forward_pair(self._h, B, T, _ptr(e2), _ptr(a2), _ptr(y), _ptr(s2),
                                               _ptr(saved), _stream(e2.device)))
        return y, s2, saved

    def backward_pair(self, g: torch.Tensor, a2: torch.Tensor, e2: torch.Tensor, saved: torch.Tensor,
                      s2: Optional[torch.Tensor] = None, need_e: bool = True, need_a: bool = True):
        """Shared upstream gradient g = dL/dy [B,T] -> (grad_e2 [2,B,T], grad_a2 [2,B,T,M])."""
        _need(g, "g", torch.float32, 2)
        B, T = g.shape
        ge2 = torch.empty_like(e2) if need_e else None
        ga2 = torch.empty_like(a2) if need_a else None
        _lib.check(_lib.load().lp_backward_pair(self._h, B, T, _ptr(g), _ptr(a2), _ptr(e2), _ptr(s2),
                                                _ptr(saved), _ptr(ge2), _ptr(ga2), _stream(g.device)))
        return ge2, ga2


class PairStepGraph:
    """A captured hipGraph of one forward + adjoint step of a filter pair on fixed buffers."""

    def __init__(self, plan: Plan, e2, a2, y, s2, saved, g, ge2, ga2, store_s: bool = False):
        self.plan = plan
        self.buffers = (e2, a2, y, s2, saved, g, ge2, ga2)  # keep alive
        _, B, T = e2.shape
        h = ctypes.c_void_p()
        torch.cuda.synchronize(e2.device)
        _lib.check(_lib.load().lp_graph_capture_pair_step(
            plan.handle, B, T, _ptr(e2), _ptr(a2), _ptr(y), _ptr(s2), _ptr(saved), _ptr(g), _ptr(ge2),
            _ptr(ga2), 1 if store_s else 0, ctypes.byref(h)))
        self._h = h

    def launch(self, stream: Optional[torch.cuda.Stream] = None):
        st = torch.cuda.current_stream() if stream is None else stream
        _lib.check(_lib.load().lp_graph_launch(self._h, ctypes.c_void_p(st.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().lp_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


def coef_frames_count(T: int, hop: int) -> int:
    """Frame-rate coefficient rows for a length-T signal: (T - 1) // hop + 2."""
    return int(_lib.load().lp_coef_frames_count(int(T), int(hop)))


def frames_count(T: int, hop: int) -> int:
    """Frames of the frame-wise approximation for a length-T signal: ceil(T / hop) + 3."""
    return int(_lib.load().lp_frames_count(int(T), int(hop)))


def framewise_forward(plan: "Plan", e: torch.Tensor, af: torch.Tensor, hop: int):
    """Frame-wise approximation of the filter (frames of 4 hop samples, 75 % overlap):
    e [B,T], af [B,F,M] (F = frames_count(T, hop)) -> (s [B,T], ctx for the adjoint).

    Gather the frames, filter each with its own time-invariant row (lp_forward_ti on
    the plan, whose chunk length should cover a frame), overlap-add through the
    halved Hann window.
    """
    _need(e, "e", torch.float32, 2)
    _need(af, "af", torch.float32, 3)
    B, T = e.shape
    F, W, M = frames_count(T, hop), 4 * hop, plan.M
    if af.shape != (B, F, M):
        raise ValueError(f"af must have shape {(B, F, M)}, got {tuple(af.shape)}")
    lib, st = _lib.load(), _stream(e.device)
    ef = torch.empty((B * F, W), dtype=torch.float32, device=e.device)
    _lib.check(lib.lp_frames_gather(B, T, hop, _ptr(e), _ptr(ef), 0, st))
    sf, _, saved = plan.forward_ti(ef, af.reshape(B * F, M))
    s = torch.empty_like(e)
    _lib.check(lib.lp_frames_overlap_add(B, T, hop, _ptr(sf), _ptr(s), 1, st))
    return s, (ef, sf, saved)


def framewise_backward(plan: "Plan", g: torch.Tensor, af: torch.Tensor, ctx, hop: int):
    """Adjoint of framewise_forward: returns (grad_e [B,T], grad_af [B,F,M])."""
    _need(g, "g", torch.float32, 2)
    ef, sf, saved = ctx
    B, T = g.shape
    F, W, M = frames_count(T, hop), 4 * hop, plan.M
    lib, st = _lib.load(), _stream(g.device)
    gf = torch.empty((B * F, W), dtype=torch.float32, device=g.device)
    _lib.check(lib.lp_frames_gather(B, T, hop, _ptr(g), _ptr(gf), 1, st))
    gef, gaf, _ = plan.backward_ti(gf, af.reshape(B * F, M), ef, saved, s=sf)
    ge = torch.empty_like(g)
    _lib.check(lib.lp_frames_overlap_add(B, T, hop, _ptr(gef), _ptr(ge), 0, st))
    return ge, gaf.reshape(B, F, M)
