"""Long high-resonance workload: 512 sequences x 240000 samples, order 32, poles up to 0.995.

The whole batch runs through the chunked forward and recompute adjoint on the
GPU; eight sampled sequences are copied back and compared with the float64
oracle (after screening that the oracle's output stays finite and bounded).
Inputs are bounded random-walk reflection coefficients (|k| <= 0.995) with
bandwidth expansion 0.995, built on the device by the same recipe as the host
generator.  The error of the grouped carry (transitions composed into group
matrices) and of the chained carry (LP_FLAG_CHAINED_CARRY) at the default chunk
length is reported only; a plan created for high pole radii
(LP_FLAG_HIGH_RADIUS: the chained carry over the order's longest chunks, and
an autotuner that keeps to long chunks) must meet the 1e-4 rms-relative bound
as it comes.  (On these inputs single chunk transitions of a few hundred
samples have entries in the thousands; longer chunks let the transient die
out.)
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS
from synth.device import stress_inputs
from tests.pins import rms_rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05128_amd as tv
    oracle.build(force=False)
    return tv


def _errors(tv, e, a, g, picks, chained, chunk=None, high_radius=False):
    M = a.shape[2]
    plan = tv.Plan(M, e.device, chunk, chained=chained, high_radius=high_radius)
    s, _, saved = plan.forward(e, a)
    ge, ga, _ = plan.backward(g, a, e, saved)
    plan.check_status()
    torch.cuda.synchronize()
    del saved
    worst = {}
    per_seq = []
    for b in picks:
        eb, ab, gb = (x[b:b + 1].cpu().numpy() for x in (e, a, g))
        s_ref, _ = oracle.lp_forward(eb, ab)
        assert np.all(np.isfinite(s_ref)) and np.max(np.abs(s_ref)) < 1e30, f"sequence {b} diverges"
        ge_ref, ga_ref, _ = oracle.lp_backward(gb, ab, s_ref)
        errs = {"s": rms_rel(s[b].cpu().numpy(), s_ref[0]),
                "grad_e": rms_rel(ge[b].cpu().numpy(), ge_ref[0]),
                "grad_a": rms_rel(ga[b].cpu().numpy(), ga_ref[0])}
        per_seq.append(float(f"{max(errs.values()):.3g}"))
        for k, v in errs.items():
            worst[k] = max(worst.get(k, 0.0), v)
    del s, ge, ga
    torch.cuda.empty_cache()
    return plan.chunk, worst, per_seq


def test_stress_b512_t240000_m32_sampled_sequences(tv):
    wl = WORKLOADS["stress_b512_t240000_m32"]
    B, T, M = wl.B, wl.T, wl.M
    dev = torch.device("cuda", 0)
    e, a, g = stress_inputs(B, T, M, wl.kappa, 0.995, wl.seed, dev)
    picks = np.random.default_rng(wl.seed).choice(B, 8, replace=False)
    results = {}
    for name, chained, hr in (("grouped, default L", False, False), ("chained, default L", True, False),
                              ("high-radius plan, its default L", False, True)):
        L, worst, per_seq = _errors(tv, e, a, g, picks, chained, None, hr)
        results[name] = worst
        print(f"stress B={B} T={T} M={M} {name} (L={L}): worst {worst}, per sequence {per_seq}")
    # reported, not gated: the composed (grouped) carry and mid-length chunks lose
    # accuracy on these inputs; a plan made for high pole radii (chained carry over
    # its longest chunks) meets 1e-4 without any further setting
    assert all(np.isfinite(v) for w in results.values() for v in w.values())
    assert all(v <= 1e-4 for v in results["high-radius plan, its default L"].values()), results


def test_high_radius_plan_autotunes_to_accurate_lengths(tv):
    """The autotuner of a high-radius plan keeps to chunk lengths of at least 1536
    (or the order's longest), and the chunk it picks meets 1e-4 on the stress
    inputs (a shorter slice of them: 64 sequences of 240000 samples)."""
    wl = WORKLOADS["stress_b512_t240000_m32"]
    B, T, M = 64, wl.T, wl.M
    dev = torch.device("cuda", 0)
    e, a, g = stress_inputs(B, T, M, wl.kappa, 0.995, wl.seed, dev)
    plan = tv.Plan(M, dev, high_radius=True)
    longest = plan.chunk
    tune = plan.autotune(B, T, reps=1, cache=False)
    print(f"high-radius plan M={M}: longest chunk {longest}, autotuned {tune}")
    assert min(1536, longest) <= tune["chunk"] <= longest and tune["chunk"] % M == 0
    picks = np.random.default_rng(wl.seed + 1).choice(B, 4, replace=False)
    L, worst, per_seq = _errors(tv, e, a, g, picks, False, tune["chunk"], True)
    print(f"high-radius plan, autotuned L={L}: worst {worst}, per sequence {per_seq}")
    assert all(v <= 1e-4 for v in worst.values()), worst
