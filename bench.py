#!/usr/bin/env python3
"""Throughput of the time-varying LP filter, forward + adjoint, on one MI355X.

One step = chunked forward (s = LP_a(e), Eq. 6) + chunked adjoint with per-chunk
recomputation of s (Eqs. 12-13) over one batch of the training-shape workload:
B = 64 sequences of T = 48000 samples (2 s at 24 kHz), order M = 22, synthetic
speech-shaped inputs (reflection coefficients drawn every 240 samples,
interpolated, converted by the step-up recursion).  Inputs are resident in HBM
before timing starts; two input sets alternate so that one step's inputs are
not left in the last-level cache by the previous step.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd filtered samples/s at M=22 (chunked vs sequential); serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, published
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published


# HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors from a
# plain 256 MiB device copy) of the four row-streaming kernels for the training workload,
# per chunk length, measured with the chained carry.  These kernels are the same launches
# in both carry modes (the carry mode only changes the carry kernels between them).  Valid
# only for the kernel sources (hash below) they were measured with, otherwise null.
TRAFFIC = {
    "sources_sha256": "0518989db867124d6318499a219066429b1230d358cb15d2f5e5c18762ecf01c",
    "measured_with_carry": "chained",
    "bytes_by_chunk": {
        396: {"fwd_scan": 319674597, "fwd_emit": 320343252, "bwd_scan": 627050543, "bwd_emit": 582741050},
        418: {"fwd_scan": 315566905, "fwd_emit": 319093989, "bwd_scan": 625221550, "bwd_emit": 582673912},
        440: {"fwd_scan": 315229279, "fwd_emit": 314743010, "bwd_scan": 612850460, "bwd_emit": 581682640},
    },
}


def kernel_sources_sha256() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2406_05128_amd", "csrc", "*"))):
        if os.path.basename(f) in ("tvlp_serve.hip", "tvlp_sf.hip"):  # no LP kernels in these
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, chunk: int):
    if kernel_sources_sha256() != TRAFFIC["sources_sha256"]:
        return None
    return TRAFFIC["bytes_by_chunk"].get(chunk, {}).get(kernel)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(name: str, B: int, T: int, M: int, L: int) -> float:
    """Algorithmic HBM bytes credited to one launch of each kernel.

    One step must move 4(3M+5) bytes per sample: the forward reads e and a and
    writes s (4M+8), the adjoint with recomputed s reads g, e and a and writes
    grad_e and grad_a (8M+12).  Each of these tensors is credited once, to the
    first kernel that moves it: fwd_scan reads e and a of the chunks that carry a
    transition, fwd_emit reads e and a of each sequence's last chunk and writes s,
    bwd_scan reads g, e and a, bwd_emit writes grad_e and grad_a.  What a kernel
    moves beyond that (the forward's second pass over e and a, the adjoint's
    further passes over a, the recompute of s, chunk states and transitions) is
    overhead: it appears in the measured traffic, never here.  Summed over the
    kernels the figures are 4(3M+5) B T.
    """
    n = B * T
    C = -(-T // L)
    n_full = B * (C - 1) * L  # samples in chunks that carry a transition
    row = 4 * M
    table = {
        "fwd_scan": n_full * (4 + row),                  # e, a (transition-carrying chunks)
        "fwd_emit": (n - n_full) * (4 + row) + n * 4,    # e, a (last chunks); s
        "bwd_scan": n * (4 + 4 + row),                   # g, e, a
        "bwd_emit": n * (4 + row),                       # grad_e, grad_a
    }
    return float(table.get(name, 0.0))


def kernel_design_bytes(name: str, B: int, T: int, M: int, L: int) -> float:
    """HBM bytes each kernel of the current design moves by construction (the
    algorithmic bytes plus the re-reads its pass structure needs; chunk-state
    side arrays excluded): what the hardware counters are checked against."""
    n = B * T
    C = -(-T // L)
    n_full = B * (C - 1) * L
    row = 4 * M
    table = {
        "fwd_scan": n_full * (4 + row),                  # e, a
        "fwd_emit": n * (4 + row + 4),                   # e, a; s
        # adjoint local scan (g, a) and, in the same launch, s recomputed (e, a; s to workspace)
        "bwd_scan": n * (4 + row) + n * (4 + row + 4),
        "bwd_emit": n * (4 + 4 + row) + n * (4 + row),   # g, s, a; grad_e, grad_a
    }
    return float(table.get(name, 0.0))


def step_bytes(B: int, T: int, M: int) -> float:
    """Algorithmic bytes of one forward + recompute-adjoint step, 4(3M+5) per sample."""
    return float(B * T * 4 * (3 * M + 5))


def serve_bench(tv, n_req: int, seed: int, slots: int, budget_gib: float, batch: int,
                timeout_ms: float = 50.0, small_budget_mb: int = 256):
    """Serving workload: open-loop Poisson arrivals (200 req/s, lengths U(12000,
    240000), M = 22, forward only, host-pinned e/a/s) through

    * the native continuous-batching server with a `budget_gib` arena, and again
      with a `small_budget_mb` arena (admission by HBM budget under pressure);
    * a padded fixed-batch baseline fed the same arrival stream: up to `batch`
      requests, launched when the batch is full or its oldest request has waited
      `timeout_ms`, padded to the batch's longest request and run as one uniform
      lp_forward (packing, copies and compute in the request's latency).

    Each run reports p50/p99 of the host latency (arrival to result in host
    memory) and of the device time (server: a job's first slice to its last;
    padded: the batch's filter launches), and the useful samples per second.
    """
    import collections

    import numpy as np
    import torch
    from synth import make_coeffs, make_excitation, poisson_requests

    M = 22
    rng = np.random.default_rng(seed)
    arrivals, lengths = poisson_requests(rng, n_req, 200.0, 12000, 240000)
    pool_T = 600_000
    log(f"serve: coefficient pool of {pool_T} samples")
    a_pool = torch.from_numpy(make_coeffs(rng, 1, pool_T, M, 0.9)[0]).pin_memory()
    e_pool = torch.from_numpy(make_excitation(rng, 1, pool_T)[0]).pin_memory()
    offs = [int(rng.integers(0, pool_T - int(T) + 1)) for T in lengths]
    outs = [torch.empty(int(T), dtype=torch.float32, pin_memory=True) for T in lengths]
    useful = float(np.sum(lengths))

    def pct(x):
        x = np.asarray(x, dtype=np.float64)
        return {"p50_ms": round(float(np.percentile(x, 50)), 3), "p99_ms": round(float(np.percentile(x, 99)), 3),
                "mean_ms": round(float(x.mean()), 3)}

    def continuous(budget_bytes: int, label: str):
        with tv.Server(M, budget_bytes, max_slots=slots) as srv:
            t = srv.submit(e_pool[:24000], a_pool[:24000])  # warm the kernels and the scheduler
            srv.wait(t, 60.0)
            log(f"serve ({label}): {n_req} requests at 200/s, {slots} slots, {budget_bytes / 2**20:.0f} MiB arena")
            tickets = []
            t0 = time.perf_counter()
            for k in range(n_req):
                delay = float(arrivals[k]) - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                o, T = offs[k], int(lengths[k])
                tickets.append(srv.submit(e_pool[o:o + T], a_pool[o:o + T], out=outs[k]))
            done = [srv.wait(tk, 120.0, device_time=True) for tk in tickets]
            wall = time.perf_counter() - t0
            st = srv.stats()
        return {"host": pct([d[1] for d in done]), "device": pct([d[2] for d in done]),
                "arena_MiB": round(budget_bytes / 2**20, 1), "iterations": st["iterations"],
                "samples_per_s": round(useful / wall, 1), "wall_s": round(wall, 3)}

    res = {"requests": n_req, "rate_hz": 200.0, "len_range": [12000, 240000], "M": M, "slots": slots,
           "offered_samples_per_s": round(useful / float(arrivals[-1]), 1)}
    res["continuous"] = continuous(int(budget_gib * (1 << 30)), "large arena")
    res["continuous_small_budget"] = continuous(small_budget_mb << 20, "small arena")

    # padded fixed batches on the same arrival stream
    dev = torch.device("cuda", 0)
    plan = tv.Plan(M, dev)
    tmax = int(np.max(lengths))
    e_pad = torch.zeros((batch, tmax), dtype=torch.float32, pin_memory=True)
    a_pad = torch.zeros((batch, tmax, M), dtype=torch.float32, pin_memory=True)
    s_pad = torch.empty((batch, tmax), dtype=torch.float32, pin_memory=True)
    plan.reserve(batch, tmax)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # warm-up of the uniform path at the largest shape
    plan.forward(e_pad.to(dev), a_pad.to(dev), save=False)
    torch.cuda.synchronize()
    log(f"serve (padded): batches of {batch}, {timeout_ms} ms timeout")
    host_lat, dev_lat = [], []
    padded = 0
    queue = collections.deque()
    i = 0
    t0 = time.perf_counter()
    while i < n_req or queue:
        now = time.perf_counter() - t0
        while i < n_req and float(arrivals[i]) <= now:
            queue.append(i)
            i += 1
        if not queue:
            time.sleep(max(0.0, float(arrivals[i]) - now))
            continue
        oldest = float(arrivals[queue[0]])
        if len(queue) < batch and now - oldest < timeout_ms * 1e-3 and i < n_req:
            time.sleep(max(0.0, min(float(arrivals[i]), oldest + timeout_ms * 1e-3) - now))
            continue
        ids = [queue.popleft() for _ in range(min(batch, len(queue)))]
        Tb = int(max(lengths[j] for j in ids))
        nb = len(ids)
        e_pad[:nb, :Tb].zero_()
        a_pad[:nb, :Tb].zero_()
        for r, j in enumerate(ids):
            o, T = offs[j], int(lengths[j])
            e_pad[r, :T] = e_pool[o:o + T]
            a_pad[r, :T] = a_pool[o:o + T]
        ed = e_pad[:nb, :Tb].to(dev, non_blocking=True)
        ad = a_pad[:nb, :Tb].to(dev, non_blocking=True)
        ev0.record()
        sd, _, _ = plan.forward(ed.contiguous(), ad.contiguous(), save=False)
        ev1.record()
        s_pad[:nb, :Tb].copy_(sd, non_blocking=True)
        torch.cuda.synchronize()
        t_end = time.perf_counter() - t0
        for r, j in enumerate(ids):
            outs[j].copy_(s_pad[r, :int(lengths[j])])
            host_lat.append(1e3 * (t_end - float(arrivals[j])))
            dev_lat.append(ev0.elapsed_time(ev1))
        padded += nb * Tb
    wall = time.perf_counter() - t0
    res["padded_fixed_batch"] = {"batch": batch, "timeout_ms": timeout_ms, "host": pct(host_lat),
                                 "device": pct(dev_lat), "samples_per_s": round(useful / wall, 1),
                                 "padding_efficiency": round(useful / padded, 4), "wall_s": round(wall, 3)}
    c = res["continuous"]
    res["p50_ms"], res["p99_ms"] = c["host"]["p50_ms"], c["host"]["p99_ms"]
    return res


def time_invariant_bench(tv, B: int, T: int, M: int, L: int, steps: int, warmup: int):
    """Training shape with one coefficient row per sequence (a [B,M], Sec. 2.2):
    forward + recompute adjoint through lp_forward_ti / lp_backward_ti.

    Algorithmic bytes per sample: e, s (forward), g, e, grad_e (adjoint) = 20 B;
    the coefficient rows and their gradient are B*M floats each.
    """
    import numpy as np
    import torch
    from synth import make_excitation, make_upstream_grad, reflection_to_lpc

    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(77)
    a = np.stack([reflection_to_lpc(rng.uniform(-0.95, 0.95, size=M)) for _ in range(B)]).astype(np.float32)
    e = torch.from_numpy(make_excitation(rng, B, T)).to(dev)
    g = torch.from_numpy(make_upstream_grad(rng, B, T)).to(dev)
    a = torch.from_numpy(a).to(dev)
    plan = tv.Plan(M, dev, L)
    plan.reserve(B, T)

    def step():
        s, _, saved = plan.forward_ti(e, a)
        return plan.backward_ti(g, a, e, saved)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.set_timing(True)
    plan.reset_timings()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kern = {k: round(1e3 * v[0] / max(v[1], 1), 2) for k, v in plan.timings().items()}
    plan.set_timing(False)
    plan.check_status()
    alg = B * T * 20 + 2 * B * M * 4
    return {"workload": f"time_invariant_b{B}_t{T}_m{M}", "chunk": L, "ms_per_step": round(ms, 4),
            "samples_per_s": round(B * T / (ms * 1e-3), 1),
            "step_hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels_us": kern,
            "note": "one transition per sequence (companion-matrix power by repeated squaring), zero-state "
                    "chunk offsets by a rerun, chained carry; coefficient rows read with step 0 by the same "
                    "chunked rerun and adjoint kernels"}


def frame_rate_bench(tv, B: int, T: int, M: int, L: int, steps: int, warmup: int, ms_samplewise: float,
                     fixed_chunk: int = 0):
    """Training shape with frame-rate LP coefficients (Sec. 4.3: one row per
    240-sample frame, linearly upsampled to the sample rate) interpolated inside
    the kernels: forward + recompute adjoint through lp_forward_frames /
    lp_backward_frames, giving dL/de and dL/dA [B,F,M].

    Algorithmic bytes per sample: e, s (forward), g, e, grad_e (adjoint) = 20 B;
    the frame rows and their gradient are B*F*M floats each.  Agreement with the
    per-sample path is checked on 4 sequences whose rows are upsampled on the host
    (numpy.interp) and fed to lp_forward / lp_backward.
    """
    import numpy as np
    import torch
    from synth import make_excitation, make_upstream_grad, reflection_to_lpc

    hop = 240
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(78)
    F = tv.coef_frames_count(T, hop)
    # bounded random walk of the reflection coefficients per frame (neighbouring
    # frames close enough that interpolated LPCs stay stable), bandwidth 0.98
    k = np.empty((B, F, M))
    k[:, 0] = rng.uniform(-0.95, 0.95, size=(B, M))
    dk = rng.normal(0.0, 0.01, size=(B, F, M))
    for f in range(1, F):
        k[:, f] = np.clip(k[:, f - 1] + dk[:, f], -0.95, 0.95)
    A_h = (reflection_to_lpc(k) * 0.98 ** np.arange(1, M + 1)).astype(np.float32)
    e_h = make_excitation(rng, B, T)
    g_h = make_upstream_grad(rng, B, T)
    A, e, g = (torch.from_numpy(x).to(dev) for x in (A_h, e_h, g_h))

    def step_with(p_):
        s, _, saved = p_.forward_frames(e, A, hop)
        return p_.backward_frames(g, A, hop, e, saved)

    # chunk length: a short sweep around the per-sample choice (the frame-rate kernels
    # hold more LDS per wave, which moves the occupancy steps)
    sweep = {}
    cands = [fixed_chunk] if fixed_chunk else sorted({L} | {k * M for k in range(max(1, (L - 5 * M) // M),
                                                                                  (L + 6 * M) // M + 1)})
    for Lc in cands:
        try:
            pc = tv.Plan(M, dev, Lc)
            for _ in range(2):
                step_with(pc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                step_with(pc)
            torch.cuda.synchronize()
            sweep[Lc] = round((time.perf_counter() - t0) * 1e3 / 5, 4)
        except Exception as ex:  # chunk lengths whose staged frame rows do not fit
            log(f"frame-rate: chunk {Lc} skipped ({ex})")
    L = min(sweep, key=sweep.get)
    plan = tv.Plan(M, dev, L)

    def step():
        return step_with(plan)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.set_timing(True)
    plan.reset_timings()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kern = {k: round(1e3 * v[0] / max(v[1], 1), 2) for k, v in plan.timings().items()}
    plan.set_timing(False)
    # agreement with the per-sample path on rows upsampled on the host
    nb = 4
    x = np.arange(T)
    a_h = np.empty((nb, T, M), np.float32)
    for b in range(nb):
        for i in range(M):
            a_h[b, :, i] = np.interp(x, np.arange(F) * hop, A_h[b, :, i])
    a4 = torch.from_numpy(a_h).to(dev)
    s_f, _, sv_f = plan.forward_frames(e[:nb].contiguous(), A[:nb].contiguous(), hop)
    ge_f, _, _ = plan.backward_frames(g[:nb].contiguous(), A[:nb].contiguous(), hop, e[:nb].contiguous(), sv_f)
    s_p, _, sv_p = plan.forward(e[:nb].contiguous(), a4)
    ge_p, _, _ = plan.backward(g[:nb].contiguous(), a4, e[:nb].contiguous(), sv_p, need_a=False)
    torch.cuda.synchronize()
    plan.check_status()

    def rel(x_, r_):
        d = x_.double() - r_.double()
        return float(torch.sqrt((d * d).mean(dim=1) / (r_.double() ** 2).mean(dim=1)).max())

    alg = B * T * 20 + 2 * B * F * M * 4
    return {"workload": f"frame_rate_b{B}_t{T}_m{M}_hop{hop}", "frames": F, "chunk": L, "chunk_sweep_ms": sweep,
            "ms_per_step": round(ms, 4), "samples_per_s": round(B * T / (ms * 1e-3), 1),
            "vs_samplewise_time": round(ms / ms_samplewise, 3),
            "step_hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels_us": kern,
            "max_rms_rel_diff_vs_per_sample_rows_4seq": {"s": round(rel(s_f, s_p), 9),
                                                         "grad_e": round(rel(ge_f, ge_p), 9)},
            "inputs": "reflection coefficients per frame as a bounded random walk (|k| <= 0.95, step sd 0.01), "
                      "step-up at the frame rate, a_i scaled by 0.98^i",
            "note": "rows interpolated in LDS by the ring producers (no [B,T,M] array read or written); "
                    "dL/dA from per-chunk float64 shares summed per frame"}


def sf_synth_bench(tv, B: int, T: int, M: int, steps: int, warmup: int):
    """The source-filter synthesiser of Eq. 5 around the LP filter on the training
    shape: pulse train plus frame-wise FIR filtered noise (510 taps per 240-sample
    frame, the length of a 256-bin frequency response), input gain, frame-rate LP
    (M = 22), 128-tap output FIR; forward + adjoint of every parameter.  Stages
    are timed with events on the stream; the noise filter and the output FIR are
    float32 FMA streams (2 FLOP per tap and sample) reported against the fp32
    vector peak."""
    import numpy as np
    import torch
    from synth import make_excitation, make_upstream_grad, pulse_train, reflection_to_lpc
    from paper_2406_05128_amd import _lib
    from paper_2406_05128_amd.ops import _ptr, _stream

    hop, K, K2 = 240, 510, 128
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(91)
    F = tv.coef_frames_count(T, hop)
    k = np.empty((B, F, M))
    k[:, 0] = rng.uniform(-0.95, 0.95, size=(B, M))
    dk = rng.normal(0.0, 0.01, size=(B, F, M))
    for f in range(1, F):
        k[:, f] = np.clip(k[:, f - 1] + dk[:, f], -0.95, 0.95)
    A = (reflection_to_lpc(k) * 0.98 ** np.arange(1, M + 1)).astype(np.float32)
    p = pulse_train(rng, B, T)
    n = make_excitation(rng, B, T)
    C = (rng.standard_normal((B, F, K)) / np.sqrt(K)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, size=(B, F)).astype(np.float32)
    h = (rng.standard_normal(K2) / np.sqrt(K2)).astype(np.float32)
    gy = make_upstream_grad(rng, B, T)
    p, n, C, gain, A, h, gy = (torch.from_numpy(x).to(dev) for x in (p, n, C, gain, A, h, gy))
    syn = tv.SFSynth(M, hop, K, K2, dev)

    def step():
        y, ctx = syn.forward(p, n, C, gain, A, h)
        return syn.backward(gy, ctx)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # the source and FIR kernels alone, events on the stream they are launched on
    lib, st = _lib.load(), _stream(dev)
    u, x, y = (torch.empty_like(p) for _ in range(3))

    def timed(fn, reps=5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3  # us

    us_src = timed(lambda: lib.lp_sf_source(B, T, hop, K, _ptr(p), _ptr(n), _ptr(C), _ptr(gain), _ptr(u), _ptr(x), st))
    us_fir = timed(lambda: lib.lp_fir(B, T, K2, _ptr(x), _ptr(h), _ptr(y), st))
    gC, gg, gs, gh = torch.empty_like(C), torch.empty_like(gain), torch.empty_like(p), torch.empty_like(h)
    work = torch.empty(lib.lp_fir_adjoint_work_bytes(B, T, K2), dtype=torch.uint8, device=dev)
    us_src_adj = timed(lambda: lib.lp_sf_source_adjoint(B, T, hop, K, _ptr(gy), _ptr(u), _ptr(n), _ptr(gain),
                                                        _ptr(gs), _ptr(gC), _ptr(gg), st))
    us_fir_adj = timed(lambda: lib.lp_fir_adjoint(B, T, K2, _ptr(gy), _ptr(x), _ptr(h), _ptr(gs), _ptr(gh),
                                                  _ptr(work), st))
    flops_src = 2.0 * B * T * K
    flops_fir = 2.0 * B * T * K2
    return {"workload": f"sf_synth_b{B}_t{T}_m{M}_hop{hop}_k{K}_fir{K2}", "ms_per_step": round(ms, 4),
            "samples_per_s": round(B * T / (ms * 1e-3), 1),
            "kernels_us": {"source_fir_noise": round(us_src, 2), "output_fir": round(us_fir, 2),
                           "source_adjoint": round(us_src_adj, 2), "output_fir_adjoint": round(us_fir_adj, 2)},
            "source_fir_noise_TFLOPs_f32": round(flops_src / (us_src * 1e-6) / 1e12, 2),
            "output_fir_TFLOPs_f32": round(flops_fir / (us_fir * 1e-6) / 1e12, 2),
            "source_adjoint_TFLOPs_f32": round(flops_src / (us_src_adj * 1e-6) / 1e12, 2),
            "output_fir_adjoint_TFLOPs_f32": round(2 * flops_fir / (us_fir_adj * 1e-6) / 1e12, 2),
            "fp32_vector_peak_TFLOPs": FP32_PEAK_TFLOPS,
            "note": "one step = source, frame-rate LP, output FIR and the adjoint of each; LP parts as in the "
                    "frame-rate section"}


def framewise_bench(tv, sets, B: int, T: int, M: int, steps: int, warmup: int, ms_samplewise: float):
    """The frame-wise approximation (hop 240 = 10 ms at 24 kHz, frames of 960 samples,
    75 % overlap) on the training shape: frames filtered with the coefficient row
    at their centre, overlap-added; forward + adjoint timed like the sample-wise
    step. Its output is compared with the sample-wise filter on the same inputs
    (coefficients bandwidth-expanded to pole radius <= 0.98) for two coefficient
    families: the timed tracks, whose filter is redrawn independently every hop
    so a 960-sample frame spans four unrelated filters, and a random walk of the
    reflection coefficients (slow drift, 8 sequences)."""
    import numpy as np
    import torch
    from synth.inputs import make_coeffs, make_excitation
    hop = 240
    dev = torch.device("cuda", 0)
    e, a, g = sets[0]
    # bandwidth-expanded rows (a_i 0.98^i, pole radius <= 0.98): the literal rows
    # resonate for far longer than a frame, where the approximation has no meaning
    a = (a * torch.tensor([0.98 ** (i + 1) for i in range(M)], dtype=torch.float32, device=dev)).contiguous()
    F = tv.frames_count(T, hop)
    centres = torch.clamp(torch.arange(F, device=dev) * hop - hop, 0, T - 1)
    af = a[:, centres, :].contiguous()  # [B, F, M]
    L = -(-4 * hop // M) * M  # one chunk per frame
    plan = tv.Plan(M, dev, L)

    def step():
        s, ctx = tv.framewise_forward(plan, e, af, hop)
        return s, tv.framewise_backward(plan, g, af, ctx, hop)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ref = tv.Plan(M, dev)

    def rms_rel(e_, a_):
        af_ = a_[:, centres, :].contiguous()
        s_fw, _ = tv.framewise_forward(plan, e_, af_, hop)
        s_sw, _, _ = ref.forward(e_, a_)
        d = s_fw.double() - s_sw.double()
        return float(torch.sqrt((d * d).mean(dim=1) / (s_sw.double() ** 2).mean(dim=1)).median())

    err_iid = rms_rel(e, a)
    rng = np.random.default_rng(5)
    a_rw = torch.from_numpy(make_coeffs(rng, 8, T, M, 0.95, 0.98, "randomwalk")).to(dev)
    e_rw = torch.from_numpy(make_excitation(rng, 8, T)).to(dev)
    err_rw = rms_rel(e_rw, a_rw)
    torch.cuda.synchronize()
    plan.check_status()
    return {"workload": f"framewise_b{B}_t{T}_m{M}_hop{hop}", "frames": F, "frame_len": 4 * hop,
            "chunk": L, "ms_per_step": round(ms, 4), "samples_per_s": round(B * T / (ms * 1e-3), 1),
            "vs_samplewise_time": round(ms / ms_samplewise, 3),
            "inputs": "a_i scaled by 0.98^i (pole radius <= 0.98)",
            "rms_rel_diff_vs_samplewise_median": {"training_tracks_redrawn_every_hop": round(err_iid, 5),
                                                   "random_walk_reflections_8seq": round(err_rw, 5)},
            "note": "frames filtered sample-serially inside each chunk like the sample-wise path; 4x the "
                    "samples (75 % overlap) and no transitions to carry"}


def stress_bench(tv, steps: int):
    """Long high-resonance workload (512 x 240000, M = 32, |k| <= 0.995, gamma 0.995).

    A plan made for high pole radii (LP_FLAG_HIGH_RADIUS: chained carry, chunk
    length autotuned among the lengths long enough for its accuracy); reports
    fwd+adjoint throughput at the autotuned chunk, and the error against the
    float64 oracle of each of 8 sampled sequences.
    """
    import numpy as np
    import torch
    import oracle
    from synth import WORKLOADS
    from synth.device import stress_inputs

    wl = WORKLOADS["stress_b512_t240000_m32"]
    B, T, M = wl.B, wl.T, wl.M
    dev = torch.device("cuda", 0)
    log(f"stress: building inputs B={B} T={T} M={M} on the device")
    e, a, g = stress_inputs(B, T, M, wl.kappa, 0.995, wl.seed, dev)
    plan = tv.Plan(M, dev, high_radius=True)
    tune = plan.autotune(B, T, reps=2, cache=False)
    saved = torch.empty(plan.saved_bytes(B, T), dtype=torch.uint8, device=dev)
    s = torch.empty_like(e)

    def step():
        plan.forward(e, a, out=s, saved_out=saved)
        return plan.backward(g, a, e, saved)

    step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        ge, ga, _ = step()
    t1.record()
    torch.cuda.synchronize()
    plan.check_status()
    ms = t0.elapsed_time(t1) / steps
    picks = np.random.default_rng(wl.seed).choice(B, 8, replace=False)
    per_seq = []
    for b in picks:
        eb, ab, gb = (x[b:b + 1].cpu().numpy() for x in (e, a, g))
        s_ref, _ = oracle.lp_forward(eb, ab)
        ge_ref, ga_ref, _ = oracle.lp_backward(gb, ab, s_ref)
        errs = {}
        for k, x, r in (("s", s[b], s_ref[0]), ("grad_e", ge[b], ge_ref[0]), ("grad_a", ga[b], ga_ref[0])):
            x = x.cpu().numpy().astype(np.float64)
            errs[k] = float(f"{np.sqrt(np.mean((x - r) ** 2)) / max(np.sqrt(np.mean(r ** 2)), 1e-300):.3g}")
        per_seq.append({"sequence": int(b), **errs})
    worst = {k: max(p[k] for p in per_seq) for k in ("s", "grad_e", "grad_a")}
    log(f"stress: {ms:.2f} ms/step at L={plan.chunk}, worst rms-rel {worst}")
    return {"workload": wl.name, "plan": "high_radius (chained carry)", "chunk": plan.chunk,
            "chunk_source": "autotuner (lengths >= 1536)", "ms_per_step": round(ms, 3),
            "samples_per_s": B * T / (ms * 1e-3),
            "autotune_timed": f"{min(B, (1 << 25) // T)} x {T} samples, best {tune['ms']:.3f} ms",
            "error_rms_rel_worst": worst, "error_rms_rel_per_sequence": per_seq}


def pair_bench(tv, steps: int, warmup: int):
    """Harmonic-plus-noise filter pair (Eq. 1): two LP filters per item, H on a
    pulse train and C on noise, B = 32 items of T = 96000 samples, M = 22, one
    upstream gradient dL/dy for y = s_H + s_C.  One step (forward of both
    filters, their sum, recompute adjoint of both) is captured once in a hipGraph
    and replayed; samples/s counts 2 B T filtered samples per step.  Per-kernel
    durations come from an eager run of the same step with per-launch events."""
    import numpy as np
    import torch
    from synth import WORKLOADS, draw_reflection_frames, make_excitation, make_upstream_grad, pulse_train
    from synth.device import coeffs_from_frames

    wl = WORKLOADS["hpn_pair_b32_t96000_m22"]
    B, T, M = wl.B, wl.T, wl.M
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(wl.seed)
    log(f"pair: building inputs B={B} T={T} M={M} (two coefficient draws, pulse train and noise)")
    a2 = torch.empty((2, B, T, M), dtype=torch.float32, device=dev)
    for f in range(2):
        a2[f].copy_(coeffs_from_frames(draw_reflection_frames(rng, B, T, M, wl.kappa, wl.family), T, 1.0, dev))
    e2d = torch.from_numpy(np.stack([pulse_train(rng, B, T), make_excitation(rng, B, T)])).to(dev)
    gd = torch.from_numpy(make_upstream_grad(rng, B, T)).to(dev)
    plan = tv.Plan(M, dev)
    # the pair runs as 2B sequences through one plan: tune for that shape
    plan.autotune(2 * B, T, reps=2, cache=False)
    L = plan.chunk
    y = torch.empty((B, T), dtype=torch.float32, device=dev)
    s2 = torch.empty_like(e2d)
    saved = torch.empty(plan.saved_bytes_pair(B, T), dtype=torch.uint8, device=dev)
    ge2 = torch.empty_like(e2d)
    ga2 = torch.empty_like(a2)
    graph = tv.PairStepGraph(plan, e2d, a2, y, s2, saved, gd, ge2, ga2)
    for _ in range(warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        graph.launch()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    graph.close()
    # per-kernel durations from the eager step (events on the launch stream)
    plan.set_timing(True)
    plan.reset_timings()
    for _ in range(steps):
        plan.forward_pair(e2d, a2, y=y, s2=s2, saved=saved)
        plan.backward_pair(gd, a2, e2d, saved)
    torch.cuda.synchronize()
    tims = plan.timings()
    plan.set_timing(False)
    n = 2 * B * T
    kernels = {name: {"avg_us": round(1e3 * tms / max(cnt, 1), 2), "launches": cnt}
               for name, (tms, cnt) in tims.items()}
    # per filtered sample: e, a read forward and again by the adjoint, grad_e, grad_a
    # written (3M+3 words); y written and g read once per item, shared by its two
    # filters (1 word per filtered sample)
    alg = float(n * 4 * (3 * M + 4))
    log(f"pair: {ms:.3f} ms/step (graph replay), {n / (ms * 1e-3) / 1e9:.2f} G filtered samples/s")
    return {"workload": wl.name, "chunk": L, "chunk_source": "autotuner (2B x T)", "ms_per_step": round(ms, 4),
            "samples_per_s": n / (ms * 1e-3), "filtered_samples_per_step": n,
            "algorithmic_bytes_per_step": alg, "step_hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launch": "hipGraph replay of forward + sum + recompute adjoint", "kernels_eager": kernels}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--gamma", type=float, default=1.0,
                    help="bandwidth expansion of the coefficient tracks (1 = literal recipe)")
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--carry", choices=("auto", "chained", "grouped"), default="auto",
                    help="carry mode of the training plan (auto: the autotuner's choice, or group maps with --chunk)")
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seq-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--no-ti", action="store_true", help="skip the time-invariant coefficient section")
    ap.add_argument("--no-framewise", action="store_true", help="skip the frame-wise approximation section")
    ap.add_argument("--no-frame-rate", action="store_true", help="skip the frame-rate coefficient section")
    ap.add_argument("--no-sf", action="store_true", help="skip the source-filter synthesiser section")
    ap.add_argument("--no-pair", action="store_true", help="skip the harmonic-plus-noise filter pair section")
    ap.add_argument("--frame-rate-chunk", type=int, default=0,
                    help="chunk length of the frame-rate section (default: a short sweep)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (hardware-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path shards "
              "over sequences with no communication, but this build runs and reports a single GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2406_05128_amd as tv
    from synth import workload, WORKLOADS

    wl = WORKLOADS["train_b64_t48000_m22"]
    B, T, M = wl.B, wl.T, wl.M
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    log(f"generating inputs B={B} T={T} M={M} gamma={args.gamma}")
    t0 = time.time()
    e_np, a_np, g_np = workload(wl.name, gamma=args.gamma)
    log(f"inputs ready in {time.time() - t0:.1f}s")
    sets = []
    e0 = torch.from_numpy(e_np).to(dev)
    a0 = torch.from_numpy(a_np).to(dev)
    g0 = torch.from_numpy(g_np).to(dev)
    sets.append((e0, a0, g0))
    # second, distinct-address input set: the batch rolled by one sequence
    sets.append((e0.roll(1, 0).contiguous(), a0.roll(1, 0).contiguous(), g0.roll(1, 0).contiguous()))
    torch.cuda.synchronize()

    plan = tv.Plan(M, dev, args.chunk)
    if args.carry != "auto":
        plan.set_carry(args.carry == "chained")
    tune = None
    if args.chunk is None:
        # chunk length picked by the autotuner (fresh measurement, not the cache)
        tune = plan.autotune(B, T, reps=3, cache=False)
        log(f"autotuned chunk L={tune['chunk']}, {'chained' if tune['chained'] else 'grouped'} carry "
            f"({tune['ms']:.3f} ms/step on its stand-in inputs)")
    L = plan.chunk
    plan.reserve(B, T)
    saved = [torch.empty(plan.saved_bytes(B, T), dtype=torch.uint8, device=dev) for _ in sets]
    s_out = [torch.empty((B, T), dtype=torch.float32, device=dev) for _ in sets]

    def step(i):
        e, a, g = sets[i % 2]
        # forward fills the saved chunk states; the backward recomputes s per chunk from them
        plan.forward(e, a, out=s_out[i % 2], saved_out=saved[i % 2])
        return plan.backward(g, a, e, saved[i % 2], s=None)

    log(f"warmup {args.warmup} steps (chunk L={L})")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    log(f"timing {args.steps} steps")
    start.record()
    for i in range(args.steps):
        step(i)
    stop.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(stop) / args.steps
    value = B * T / (ms_step * 1e-3)
    log(f"chunked fwd+bwd: {ms_step:.3f} ms/step, {value / 1e9:.3f} G samples/s")

    # per-kernel durations: the same timed loop with per-launch hipEvents on the launch stream
    plan.set_timing(True)
    plan.reset_timings()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    tims = plan.timings()
    plan.set_timing(False)
    kernels = {}
    for name, (ms, n) in tims.items():
        avg_us = 1e3 * ms / max(n, 1)
        by = kernel_bytes(name, B, T, M, L)
        tr = measured_traffic(name, L)  # HBM bytes per launch from the counters, or None
        kernels[name] = {"avg_us": round(avg_us, 2), "launches": n,
                         "alg_bytes": by or None,
                         "alg_GBps": round(by / (avg_us * 1e-6) / 1e9, 1) if by else None,
                         "traffic": tr,
                         "traffic_GBps": round(tr / (avg_us * 1e-6) / 1e9, 1) if tr else None}
    # the path is bound by HBM (a scan with no dense contraction): the roofline names the
    # kernel with the longest average launch, against the HBM peak, with its share of the
    # step's algorithmic bytes
    dominant = max(tims, key=lambda k: tims[k][0] / max(tims[k][1], 1)) if tims else None
    roofline = None
    if dominant:
        d = kernels[dominant]
        by = kernel_bytes(dominant, B, T, M, L)
        ach = by / (d["avg_us"] * 1e-6) / 1e9
        traffic = measured_traffic(dominant, L)
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "algorithmic_bytes": by,
                    "traffic_over_alg": round(traffic / by, 3) if traffic and by else None}
    total_alg = step_bytes(B, T, M)
    step_frac = total_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    sequential = None
    if not args.no_sequential:
        log("sequential one-thread-per-sequence baseline")
        e, a, g = sets[0]
        s, _ = tv.forward_plain(e, a)
        tv.backward_plain(g, a, s)
        torch.cuda.synchronize()
        st0 = torch.cuda.Event(enable_timing=True)
        st1 = torch.cuda.Event(enable_timing=True)
        st0.record()
        for _ in range(args.seq_steps):
            s, _ = tv.forward_plain(e, a)
            tv.backward_plain(g, a, s)
        st1.record()
        torch.cuda.synchronize()
        ms_seq = st0.elapsed_time(st1) / args.seq_steps
        sequential = {"ms_per_step": round(ms_seq, 3), "value": B * T / (ms_seq * 1e-3),
                      "speedup_chunked": round(ms_seq / ms_step, 2)}
        log(f"sequential: {ms_seq:.2f} ms/step")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # the whole batch through the float64 oracle (forward + adjoint incl. grad_a), repeated
        # until about 10 s of host time have been spent
        log(f"CPU float64 oracle on the full batch, {oracle.num_threads()} threads")
        passes = 0
        t0 = time.time()
        while True:
            s_ref, _ = oracle.lp_forward(e_np, a_np)
            oracle.lp_backward(g_np, a_np, s_ref)
            passes += 1
            dt = time.time() - t0
            if dt >= args.cpu_seconds:
                break
        cpu = {"value": passes * B * T / dt, "unit": "samples/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{passes} passes over the full batch (B={B}, T={T}, M={M}), forward + adjoint "
                         f"incl. grad_a, float64, {dt:.1f} s"}
        log(f"oracle: {passes} passes in {dt:.1f} s")

    if args.copy_probe_mb > 0:
        # a plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the counters of the filter kernels
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {args.copy_probe_mb} MiB")
        del src, dst

    ti = None
    if not args.no_ti:
        log("time-invariant coefficients (a [B,M])")
        ti = time_invariant_bench(tv, B, T, M, L, args.steps, args.warmup)
        log(f"time-invariant: {ti['ms_per_step']:.3f} ms/step")
        torch.cuda.empty_cache()

    frame_rate = None
    if not args.no_frame_rate:
        log("frame-rate coefficients (hop 240, interpolated in the kernels)")
        frame_rate = frame_rate_bench(tv, B, T, M, L, args.steps, args.warmup, ms_step, args.frame_rate_chunk)
        log(f"frame-rate: {frame_rate['ms_per_step']:.3f} ms/step")
        torch.cuda.empty_cache()

    sf = None
    if not args.no_sf:
        log("source-filter synthesiser (Eq. 5) around the frame-rate LP")
        sf = sf_synth_bench(tv, B, T, M, args.steps, args.warmup)
        log(f"sf synthesiser: {sf['ms_per_step']:.3f} ms/step")
        torch.cuda.empty_cache()

    framewise = None
    if not args.no_framewise:
        log("frame-wise approximation (hop 240, 75 % overlap)")
        framewise = framewise_bench(tv, sets, B, T, M, args.steps, args.warmup, ms_step)
        log(f"frame-wise: {framewise['ms_per_step']:.3f} ms/step, median rms-rel difference to sample-wise "
            f"{framewise['rms_rel_diff_vs_samplewise_median']}")
        torch.cuda.empty_cache()

    stress = None
    if not args.no_stress:
        stress = stress_bench(tv, 3)
        torch.cuda.empty_cache()

    pair = None
    if not args.no_pair:
        log("harmonic-plus-noise filter pair (B=32, T=96000, graph replay)")
        pair = pair_bench(tv, args.steps, args.warmup)
        torch.cuda.empty_cache()

    serve = None
    if not args.no_serve:
        serve = serve_bench(tv, args.serve_requests, 2024, args.serve_slots, 4.0, args.serve_batch)
        log(f"serve: p50 {serve['p50_ms']} ms, p99 {serve['p99_ms']} ms (continuous batching); padded batches "
            f"p50 {serve['padded_fixed_batch']['host']['p50_ms']} ms, p99 {serve['padded_fixed_batch']['host']['p99_ms']} ms")

    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 io, f64 arithmetic", "data": "synthetic",
        "config": {"workload": wl.name, "B": B, "T": T, "M": M, "chunk": L,
                   "carry": "chained" if plan.chained else "group maps",
                   "chunk_source": "autotuner" if tune else "--chunk",
                   "inputs": f"reflection-coefficient tracks, 240-sample hop, gamma={args.gamma}",
                   "backward": "recompute s per chunk from saved float64 chunk states"},
        "step_hbm_frac": round(step_frac, 4),
        "roofline": roofline,
        "kernels": kernels,
        "sequential": sequential,
        "cpu_baseline": cpu,
        "serve": serve,
        "stress": stress,
        "pair": pair,
        "time_invariant": ti,
        "frame_rate": frame_rate,
        "sf_synth": sf,
        "framewise": framewise,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
