"""Long high-resonance workload: 512 sequences x 240000 samples, order 32, poles up to 0.995.

The whole batch runs through the chunked forward and recompute adjoint on the
GPU; eight sampled sequences are copied back and compared with the float64
oracle (after screening that the oracle's output stays finite and bounded).
Inputs are bounded random-walk reflection coefficients (|k| <= 0.995) with
bandwidth expansion 0.995, built on the device by the same recipe as the host
generator.  The error of the grouped carry (transitions composed into group
matrices) and of the chained carry (LP_FLAG_CHAINED_CARRY) at the default chunk
length is reported only; the chained carry with 2048-sample chunks, the
configuration recommended for such inputs, must meet the 1e-4 rms-relative
bound.  (On these inputs single chunk transitions of a few hundred samples have
entries in the thousands; longer chunks let the transient die out.)
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


def _errors(tv, e, a, g, picks, chained, chunk=None):
    M = a.shape[2]
    plan = tv.Plan(M, e.device, chunk, chained=chained)
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
    for name, chained, chunk in (("grouped, default L", False, None), ("chained, default L", True, None),
                                 ("chained, L=2048", True, 2048)):
        L, worst, per_seq = _errors(tv, e, a, g, picks, chained, chunk)
        results[name] = worst
        print(f"stress B={B} T={T} M={M} {name} (L={L}): worst {worst}, per sequence {per_seq}")
    # reported, not gated: the composed (grouped) carry and mid-length chunks lose
    # accuracy on these inputs; the chained carry over 2048-sample chunks meets 1e-4
    assert all(np.isfinite(v) for w in results.values() for v in w.values())
    assert all(v <= 1e-4 for v in results["chained, L=2048"].values()), results
