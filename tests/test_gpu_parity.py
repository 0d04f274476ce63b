"""HIP path vs the float64 oracle, element by element, through the C ABI.

Tolerance (stated by the method's accuracy target): per sequence and per tensor,
rms(x - x_ref) / rms(x_ref) <= 1e-4 for inputs whose frozen pole radius is at
most 0.98 (bandwidth-expanded "gated" inputs).  The kernels compute in float64
internally, so observed errors are ~1e-7 (float32 output rounding).
"""
import numpy as np
import pytest

import oracle
from synth import make_coeffs, make_excitation, make_upstream_grad, workload
from tests.pins import rms_rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def tv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05128_amd as tv
    oracle.build(force=False)
    return tv


def dev():
    return torch.device("cuda", 0)


def to_dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def host(x):
    return None if x is None else x.detach().cpu().numpy()


def per_seq_err(x, ref):
    return max(rms_rel(x[b], ref[b]) for b in range(ref.shape[0]))


def inputs(B, T, M, kappa=0.9, gamma=0.98, seed=0, family="iid"):
    rng = np.random.default_rng(seed)
    a = make_coeffs(rng, B, T, M, kappa, gamma, family)
    e = make_excitation(rng, B, T)
    g = make_upstream_grad(rng, B, T)
    return e, a, g


def check_all(tv, e, a, g, zi=None, chunk=None, store_s=False, plain=False, tol=TOL, chained=False):
    B, T, M = a.shape
    s_ref, zf_ref = oracle.lp_forward(e, a, zi)
    ge_ref, ga_ref, gz_ref = oracle.lp_backward(g, a, s_ref, zi, need_grad_zi=zi is not None)
    e_d, a_d, g_d, zi_d = to_dev(e), to_dev(a), to_dev(g), to_dev(zi)
    if plain:
        s, zf = tv.forward_plain(e_d, a_d, zi_d, want_zf=True)
        ge, ga, gz = tv.backward_plain(g_d, a_d, s, zi_d, need_zi=zi is not None)
    else:
        plan = tv.Plan(M, dev(), chunk, chained=chained)
        s, zf, saved = plan.forward(e_d, a_d, zi_d, want_zf=True)
        ge, ga, gz = plan.backward(g_d, a_d, e_d, saved, s=s if store_s else None, zi=zi_d,
                                   need_zi=zi is not None)
        plan.check_status()
    torch.cuda.synchronize()
    errs = {"s": per_seq_err(host(s), s_ref), "zf": rms_rel(host(zf), zf_ref),
            "grad_e": per_seq_err(host(ge), ge_ref), "grad_a": per_seq_err(host(ga), ga_ref)}
    if zi is not None:
        errs["grad_zi"] = rms_rel(host(gz), gz_ref)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (errs, (B, T, M, chunk))
    return errs


@pytest.mark.parametrize("plain", [False, True])
def test_small_workload_m16(tv, plain):
    e, a, g = workload("small_m16", gamma=0.98)
    print(check_all(tv, e, a, g, plain=plain))


# (B, T, M, L): T < M, T < L, ragged tails, T == L, several chunks, every compiled order class
EDGE = [
    (1, 1, 1, None), (2, 5, 16, None), (3, 100, 22, 264), (2, 264, 22, 264), (2, 265, 22, 264),
    (5, 1000, 22, 264), (1, 3000, 22, 66), (3, 1777, 16, 32), (4, 2048, 32, 64), (2, 700, 2, 8),
    (3, 513, 1, 4), (2, 999, 3, 3), (2, 640, 4, 8), (2, 777, 6, 12), (2, 800, 8, 16),
    (2, 901, 10, 20), (2, 1200, 12, 24), (2, 1300, 20, 40), (2, 1500, 24, 48),
]


@pytest.mark.parametrize("B,T,M,L", EDGE)
def test_edge_shapes_chunked(tv, B, T, M, L):
    e, a, g = inputs(B, T, M, seed=B * 1000 + T + M)
    check_all(tv, e, a, g, chunk=L)


@pytest.mark.parametrize("B,T,M,L", [(2, 5, 16, None), (3, 1000, 22, 264), (2, 901, 10, 20)])
def test_edge_shapes_plain(tv, B, T, M, L):
    e, a, g = inputs(B, T, M, seed=7 + T)
    check_all(tv, e, a, g, plain=True)


@pytest.mark.parametrize("B,T,M,L", [(3, 1000, 22, 264), (2, 7, 16, None), (2, 1024, 32, 64)])
def test_initial_state_and_state_gradient(tv, B, T, M, L):
    e, a, g = inputs(B, T, M, seed=99)
    zi = np.random.default_rng(3).standard_normal((B, M))
    check_all(tv, e, a, g, zi=zi, chunk=L)
    check_all(tv, e, a, g, zi=zi, plain=True)


# (B, T, M, L): every sequence fits one chunk (T <= L)
SINGLE = [(4, 200, 22, 264), (3, 264, 22, 264), (5, 7, 16, None), (2, 40, 8, 48), (3, 1, 1, None)]


@pytest.mark.parametrize("B,T,M,L", SINGLE)
def test_single_chunk_sequences_with_stored_s(tv, B, T, M, L):
    """Sequences that fit one chunk: the forward starts each chunk from zi (or zero)
    without a carry, and with s given the adjoint runs without its local scan and
    carries.  Both match the oracle, and the gradients equal the recompute path's
    bit for bit."""
    e, a, g = inputs(B, T, M, seed=31 + T)
    check_all(tv, e, a, g, chunk=L, store_s=True)
    zi = np.random.default_rng(5).standard_normal((B, M))
    check_all(tv, e, a, g, zi=zi, chunk=L, store_s=True)
    e_d, a_d, g_d = to_dev(e), to_dev(a), to_dev(g)
    plan = tv.Plan(M, dev(), L)
    s, _, saved = plan.forward(e_d, a_d)
    r1 = plan.backward(g_d, a_d, e_d, saved, s=None)
    r2 = plan.backward(g_d, a_d, e_d, saved, s=s)
    torch.cuda.synchronize()
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])


def test_stored_s_equals_recompute(tv):
    e, a, g = inputs(3, 5000, 22, seed=11)
    e_d, a_d, g_d = to_dev(e), to_dev(a), to_dev(g)
    plan = tv.Plan(22, dev())
    s, _, saved = plan.forward(e_d, a_d)
    r1 = plan.backward(g_d, a_d, e_d, saved, s=None)
    r2 = plan.backward(g_d, a_d, e_d, saved, s=s)
    torch.cuda.synchronize()
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])


def test_deterministic(tv):
    e, a, g = inputs(4, 6000, 22, seed=12)
    e_d, a_d, g_d = to_dev(e), to_dev(a), to_dev(g)
    plan = tv.Plan(22, dev())
    outs = []
    for _ in range(2):
        s, _, saved = plan.forward(e_d, a_d)
        ge, ga, _ = plan.backward(g_d, a_d, e_d, saved)
        outs.append((s.clone(), ge.clone(), ga.clone()))
    torch.cuda.synchronize()
    for x, y in zip(*outs):
        assert torch.equal(x, y)


def test_varlen_matches_oracle_and_alone(tv):
    rng = np.random.default_rng(21)
    M = 22
    lens = [5000, 0, 1, 264, 265, 12345, 30, 2000]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N = int(offs[-1])
    a = make_coeffs(rng, 1, N, M, 0.9, 0.98)[0]
    e = make_excitation(rng, 1, N)[0]
    g = make_upstream_grad(rng, 1, N)[0]
    plan = tv.Plan(M, dev())
    e_d, a_d, g_d, o_d = to_dev(e), to_dev(a), to_dev(g), to_dev(offs)
    s, zf, saved = plan.forward_varlen(e_d, a_d, o_d, want_zf=True)
    ge, ga, _ = plan.backward_varlen(g_d, a_d, e_d, o_d, saved)
    plan.check_status()
    torch.cuda.synchronize()
    s, ge, ga = host(s), host(ge), host(ga)
    for b in range(len(lens)):
        lo, hi = offs[b], offs[b + 1]
        if hi == lo:
            continue
        s_ref, _ = oracle.lp_forward(e[None, lo:hi], a[None, lo:hi])
        ge_ref, ga_ref, _ = oracle.lp_backward(g[None, lo:hi], a[None, lo:hi], s_ref)
        assert rms_rel(s[lo:hi], s_ref[0]) <= TOL
        assert rms_rel(ge[lo:hi], ge_ref[0]) <= TOL
        assert rms_rel(ga[lo:hi], ga_ref[0]) <= TOL
        # the same sequence alone gives bit-identical results
        s1, _, sv1 = plan.forward(e_d[lo:hi][None].contiguous(), a_d[lo:hi][None].contiguous())
        g1 = plan.backward(g_d[lo:hi][None].contiguous(), a_d[lo:hi][None].contiguous(),
                           e_d[lo:hi][None].contiguous(), sv1)
        torch.cuda.synchronize()
        assert np.array_equal(host(s1)[0], s[lo:hi])
        assert np.array_equal(host(g1[0])[0], ge[lo:hi])
        assert np.array_equal(host(g1[1])[0], ga[lo:hi])


def test_training_shape_full_size(tv):
    """B=64, T=48000, M=22 (2 s at 24 kHz), gated inputs, all sequences vs the oracle."""
    e, a, g = workload("train_b64_t48000_m22", gamma=0.98)
    errs = check_all(tv, e, a, g)
    print("train_b64_t48000_m22 gated:", errs)


@pytest.mark.parametrize("chained", [False, True])
def test_training_shape_bench_launch(tv, chained):
    """The bench's launch configuration at the training shape (L=418, which the
    autotuner picks there, in either carry mode): every sequence vs the oracle,
    gated inputs."""
    e, a, g = workload("train_b64_t48000_m22", gamma=0.98)
    errs = check_all(tv, e, a, g, chunk=418, chained=chained)
    print("train_b64_t48000_m22 L=418", "chained" if chained else "group maps", errs)


def test_training_shape_literal_inputs_reported(tv):
    """Literal (gamma = 1) inputs: error reported, not gated (poles up to ~0.9999)."""
    e, a, g = workload("train_b64_t48000_m22", gamma=1.0, B=8)
    errs = check_all(tv, e, a, g, tol=float("inf"))
    print("train literal (8 seqs):", errs)
    assert all(np.isfinite(v) for v in errs.values())


def test_autograd_function(tv):
    e, a, g = inputs(3, 3000, 16, seed=31)
    zi = np.random.default_rng(4).standard_normal((3, 16))
    e_t = to_dev(e).requires_grad_(True)
    a_t = to_dev(a).requires_grad_(True)
    zi_t = to_dev(zi).requires_grad_(True)
    s = tv.lp(e_t, a_t, zi_t)
    s.backward(to_dev(g))
    torch.cuda.synchronize()
    s_ref, _ = oracle.lp_forward(e, a, zi)
    ge_ref, ga_ref, gz_ref = oracle.lp_backward(g, a, s_ref, zi, need_grad_zi=True)
    assert per_seq_err(host(s), s_ref) <= TOL
    assert per_seq_err(host(e_t.grad), ge_ref) <= TOL
    assert per_seq_err(host(a_t.grad), ga_ref) <= TOL
    assert rms_rel(host(zi_t.grad), gz_ref) <= TOL
    # needs_input_grad honoured: only e
    e2 = to_dev(e).requires_grad_(True)
    s2 = tv.lp(e2, to_dev(a))
    s2.backward(to_dev(g))
    torch.cuda.synchronize()
    assert np.array_equal(host(e2.grad), host(e_t.grad))


def test_long_lookback_chains(tv):
    """Many groups per sequence (short chunks): look-back walks over long predecessor chains."""
    e, a, g = inputs(2, 120000, 22, seed=41)
    errs = check_all(tv, e, a, g, chunk=22)
    print("long chains (L=22, 5455 chunks/seq):", errs)


def _pair_inputs(B, T, M, seed):
    """Filter pair of the harmonic-plus-noise synthesiser (Eq. 1): H on a pulse train, C on noise."""
    from synth import pulse_train
    rng = np.random.default_rng(seed)
    a_h = make_coeffs(rng, B, T, M, 0.95, 0.98)
    a_c = make_coeffs(rng, B, T, M, 0.95, 0.98)
    e_h = pulse_train(rng, B, T)
    e_c = make_excitation(rng, B, T)
    g = make_upstream_grad(rng, B, T)
    return np.stack([e_h, e_c]), np.stack([a_h, a_c]), g


def _pair_reference(e2, a2, g):
    s_h, _ = oracle.lp_forward(e2[0], a2[0])
    s_c, _ = oracle.lp_forward(e2[1], a2[1])
    ge_h, ga_h, _ = oracle.lp_backward(g, a2[0], s_h)
    ge_c, ga_c, _ = oracle.lp_backward(g, a2[1], s_c)
    return s_h + s_c, np.stack([ge_h, ge_c]), np.stack([ga_h, ga_c])


@pytest.mark.parametrize("store_s", [False, True])
def test_filter_pair(tv, store_s):
    e2, a2, g = _pair_inputs(3, 5000, 22, seed=51)
    y_ref, ge_ref, ga_ref = _pair_reference(e2, a2, g)
    plan = tv.Plan(22, dev())
    e2d, a2d, gd = to_dev(e2), to_dev(a2), to_dev(g)
    y, s2, saved = plan.forward_pair(e2d, a2d)
    ge2, ga2 = plan.backward_pair(gd, a2d, e2d, saved, s2=s2 if store_s else None)
    plan.check_status()
    torch.cuda.synchronize()
    assert per_seq_err(host(y), y_ref) <= TOL
    for f in range(2):
        assert per_seq_err(host(ge2)[f], ge_ref[f]) <= TOL
        assert per_seq_err(host(ga2)[f], ga_ref[f]) <= TOL


def test_filter_pair_full_size(tv):
    """The harmonic-plus-noise pair at its full size (B=32, T=96000, M=22, both
    filters stacked, one upstream gradient), recompute adjoint; every item of
    both filters against the oracle."""
    B, T, M = 32, 96000, 22
    e2, a2, g = _pair_inputs(B, T, M, seed=53)
    plan = tv.Plan(M, dev())
    e2d, a2d, gd = to_dev(e2), to_dev(a2), to_dev(g)
    y, s2, saved = plan.forward_pair(e2d, a2d)
    ge2, ga2 = plan.backward_pair(gd, a2d, e2d, saved)
    plan.check_status()
    torch.cuda.synchronize()
    y_ref, ge_ref, ga_ref = _pair_reference(e2, a2, g)
    assert per_seq_err(host(y), y_ref) <= TOL
    for f in range(2):
        assert per_seq_err(host(ge2[f]), ge_ref[f]) <= TOL, f
        assert per_seq_err(host(ga2[f]), ga_ref[f]) <= TOL, f


def test_filter_pair_graph_replays(tv):
    """Captured pair step: every replay (with eager work in between) equals the eager result."""
    B, T, M = 2, 4000, 22
    e2, a2, g = _pair_inputs(B, T, M, seed=52)
    plan = tv.Plan(M, dev())
    e2d, a2d, gd = to_dev(e2), to_dev(a2), to_dev(g)
    y0, s20, sv0 = plan.forward_pair(e2d, a2d)
    ge0, ga0 = plan.backward_pair(gd, a2d, e2d, sv0)
    torch.cuda.synchronize()
    y = torch.empty_like(y0); s2 = torch.empty_like(s20); sv = torch.empty_like(sv0)
    ge2 = torch.empty_like(ge0); ga2 = torch.empty_like(ga0)
    graph = tv.PairStepGraph(plan, e2d, a2d, y, s2, sv, gd, ge2, ga2)
    for rep in range(4):
        y.fill_(float("nan")); ge2.fill_(float("nan")); ga2.fill_(float("nan"))
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(y, y0), rep
        assert torch.equal(ge2, ge0), rep
        assert torch.equal(ga2, ga0), rep
        # eager work between replays
        plan.forward_pair(e2d, a2d)
        torch.cuda.synchronize()
    plan.check_status()
    graph.close()


def test_graph_holds_the_plan_workspace(tv):
    """A captured graph keeps its plan's workspace address: while the graph exists,
    calls that would grow (move) the workspace, change the chunk length or destroy
    the plan are refused and launch nothing; calls that fit still run; after the
    graph is destroyed everything is allowed again.  (No replay ever touches a
    freed workspace: the refused calls free nothing.)"""
    from paper_2406_05128_amd import _lib
    B, T, M = 2, 4000, 22
    e2, a2, g = _pair_inputs(B, T, M, seed=54)
    plan = tv.Plan(M, dev())
    e2d, a2d, gd = to_dev(e2), to_dev(a2), to_dev(g)
    y0, s20, sv0 = plan.forward_pair(e2d, a2d)
    ge0, ga0 = plan.backward_pair(gd, a2d, e2d, sv0)
    torch.cuda.synchronize()
    y = torch.empty_like(y0); s2 = torch.empty_like(s20); sv = torch.empty_like(sv0)
    ge2 = torch.empty_like(ge0); ga2 = torch.empty_like(ga0)
    graph = tv.PairStepGraph(plan, e2d, a2d, y, s2, sv, gd, ge2, ga2)
    L0 = plan.chunk
    big_e = torch.zeros((64, 48000), dtype=torch.float32, device=dev())
    big_a = torch.zeros((64, 48000, M), dtype=torch.float32, device=dev())
    with pytest.raises(_lib.TvlpError, match="captured graph"):
        plan.forward(big_e, big_a)
    with pytest.raises(_lib.TvlpError, match="captured graph"):
        plan.set_chunk(L0 + M)
    with pytest.raises(_lib.TvlpError, match="captured graph"):
        plan.autotune(2, 4000, reps=1, cache=False)
    lib = _lib.load()
    assert lib.lp_plan_destroy(plan.handle) == _lib.LP_EINVAL
    assert plan.chunk == L0
    # a call that fits the reserved workspace still runs, and the graph still replays
    plan.forward(e2d[0], a2d[0])
    graph.launch()
    torch.cuda.synchronize()
    assert torch.equal(y, y0) and torch.equal(ge2, ge0) and torch.equal(ga2, ga0)
    graph.close()
    plan.set_chunk(L0 + M)
    s_big, _, _ = plan.forward(big_e[:4], big_a[:4])
    torch.cuda.synchronize()
    assert torch.count_nonzero(s_big).item() == 0


def test_autotuned_chunk_is_valid_and_correct(tv, tmp_path, monkeypatch):
    monkeypatch.setenv("TVLP_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    M = 22
    plan = tv.Plan(M, dev())
    res = plan.autotune(8, 5000, reps=2)
    assert not res["cached"] and res["ms"] > 0
    L = res["chunk"]
    assert L % M == 0 and M <= L <= 2048 and plan.chunk == L
    assert res["chained"] == plan.chained
    again_plan = tv.Plan(M, dev())
    again = again_plan.autotune(8, 5000)
    assert again["cached"] and again["chunk"] == L and again_plan.chained == res["chained"]
    e, a, g = inputs(3, 3001, M, seed=21)
    check_all(tv, e, a, g, chunk=L, chained=res["chained"])
    # a fixed carry mode is kept by the tuner
    fixed = tv.Plan(M, dev())
    fixed.set_carry(False)
    assert fixed.autotune(8, 5000, reps=1, cache=False)["chained"] is False and not fixed.chained


@pytest.mark.parametrize("B,T,M,L", [(3, 5000, 22, 66), (2, 9001, 32, 64), (4, 3000, 16, 32), (3, 2000, 4, 8)])
def test_chained_carry_matches_oracle(tv, B, T, M, L):
    e, a, g = inputs(B, T, M, seed=B + T + M)
    zi = np.random.default_rng(7).standard_normal((B, M)) * 0.1
    check_all(tv, e, a, g, zi=zi, chunk=L, chained=True)


def test_chained_and_grouped_carry_agree(tv):
    e, a, g = inputs(2, 20000, 22, seed=3)
    e_d, a_d, g_d = to_dev(e), to_dev(a), to_dev(g)
    out = []
    for chained in (False, True):
        plan = tv.Plan(22, dev(), 66, chained=chained)
        s, _, saved = plan.forward(e_d, a_d)
        ge, ga, _ = plan.backward(g_d, a_d, e_d, saved)
        plan.check_status()
        out.append((host(s), host(ge), host(ga)))
    for x, y in zip(*out):
        assert per_seq_err(x, y.astype(np.float64)) <= 1e-6


@pytest.mark.parametrize("M,L", [(22, 22), (22, 44), (22, 66), (22, 88), (32, 128), (32, 256), (6, 48)])
def test_unrolled_ring_region_boundaries(tv, M, L):
    """Chunk lengths around the point where the rerun and scan loops switch from
    unclamped unrolled steps to clamped ones (none, a few, most steps), with a
    ragged last chunk and both carry modes."""
    T = 3 * L + 5
    e, a, g = inputs(3, T, M, seed=M * 1000 + L)
    check_all(tv, e, a, g, chunk=L)
    check_all(tv, e, a, g, chunk=L, chained=True)


def test_misaligned_grad_a_matches_aligned(tv):
    """grad_a written through a pointer that is only 4-byte aligned takes the
    scalar store path; it must equal the (float2) aligned result bit for bit."""
    import ctypes
    from paper_2406_05128_amd import _lib
    B, T, M = 2, 3000, 22
    e, a, g = inputs(B, T, M, seed=77)
    e_d, a_d, g_d = to_dev(e), to_dev(a), to_dev(g)
    plan = tv.Plan(M, dev(), 264)
    _, _, saved = plan.forward(e_d, a_d)
    ge0, ga0, _ = plan.backward(g_d, a_d, e_d, saved)
    ge1 = torch.empty_like(g_d)
    raw = torch.empty(B * T * M + 2, dtype=torch.float32, device=dev())
    ga1 = raw[1:1 + B * T * M]  # data pointer 4 bytes past an aligned allocation
    assert ga1.data_ptr() % 8 == 4
    lib = _lib.load()
    st = torch.cuda.current_stream(dev()).cuda_stream
    rc = lib.lp_backward(plan._h, B, T, ctypes.c_void_p(g_d.data_ptr()), ctypes.c_void_p(a_d.data_ptr()),
                         ctypes.c_void_p(e_d.data_ptr()), None, None, ctypes.c_void_p(saved.data_ptr()),
                         ctypes.c_void_p(ge1.data_ptr()), ctypes.c_void_p(ga1.data_ptr()), None, None,
                         ctypes.c_void_p(st))
    assert rc == 0, lib.lp_last_error()
    torch.cuda.synchronize()
    assert torch.equal(ge0, ge1)
    assert torch.equal(ga0.reshape(-1), ga1)


def test_nonfinite_flags_only_the_affected_sequences(tv):
    """Per-sequence non-finite flags of lp_forward / lp_backward: a NaN in one
    sequence's excitation and an unstable (diverging) coefficient track in another
    flag exactly those two sequences, in the forward and in the adjoint; every
    other sequence's outputs are bit-identical to a run without the faulty
    sequences, and the flags of a clean run are all zero."""
    B, T, M = 6, 3000, 22
    e, a, g = workload("train_b64_t48000_m22", gamma=0.98, B=B, T=T)
    e_bad, a_bad = e.copy(), a.copy()
    e_bad[1, 1234] = np.nan
    a_bad[4, 100:, :] = 0.0
    a_bad[4, 100:, 0] = -1.5  # pole at 1.5 from sample 100 on: s overflows float32 within a few hundred samples
    plan = tv.Plan(M, dev(), 264)
    res = {}
    for name, (ee, aa) in (("clean", (e, a)), ("bad", (e_bad, a_bad))):
        e_d, a_d, g_d = to_dev(ee), to_dev(aa), to_dev(g)
        fl_f = torch.full((B,), 7, dtype=torch.int32, device=dev())
        fl_b = torch.full((B,), 7, dtype=torch.int32, device=dev())
        s, _, saved = plan.forward(e_d, a_d, nonfinite=fl_f)
        ge, ga, _ = plan.backward(g_d, a_d, e_d, saved, nonfinite=fl_b)
        torch.cuda.synchronize()
        res[name] = (host(s), host(ge), host(ga), fl_f.cpu().numpy(), fl_b.cpu().numpy())
    s0, ge0, ga0, f0, b0 = res["clean"]
    s1, ge1, ga1, f1, b1 = res["bad"]
    assert f0.tolist() == [0] * B and b0.tolist() == [0] * B
    assert f1.tolist() == [0, 1, 0, 0, 1, 0], f1
    assert b1.tolist() == [0, 1, 0, 0, 1, 0], b1
    assert not np.all(np.isfinite(s1[1])) and not np.all(np.isfinite(s1[4]))
    for b in (0, 2, 3, 5):
        assert np.array_equal(s1[b], s0[b]) and np.array_equal(ge1[b], ge0[b]) and np.array_equal(ga1[b], ga0[b])


def _ti_inputs(B, T, M, seed, radius=0.95):
    from tests.pins import stable_ti_coeffs
    rng = np.random.default_rng(seed)
    a = np.stack([stable_ti_coeffs(rng, M, radius) for _ in range(B)]).astype(np.float32)
    return make_excitation(rng, B, T), a, make_upstream_grad(rng, B, T)


@pytest.mark.parametrize("B,T,M,L,with_zi,store_s,chained", [
    (3, 5000, 22, 264, False, False, False),
    (2, 3001, 22, 88, True, False, False),
    (2, 4000, 16, 256, True, True, False),
    (3, 2500, 32, 128, False, False, True),
    (4, 777, 6, 48, True, False, False),
])
def test_time_invariant_matches_oracle(tv, B, T, M, L, with_zi, store_s, chained):
    """Time-invariant coefficients a [B,M]: s, grad_e, grad_a [B,M] (summed over
    time) and grad_zi against the oracle."""
    e, a, g = _ti_inputs(B, T, M, seed=B * 100 + M)
    zi = np.random.default_rng(9).standard_normal((B, M)) if with_zi else None
    s_ref, zf_ref = oracle.lp_forward_ti(e, a, zi)
    ge_ref, ga_ref, gz_ref = oracle.lp_backward_ti(g, a, s_ref, zi, need_grad_zi=with_zi)
    plan = tv.Plan(M, dev(), L, chained=chained)
    e_d, a_d, g_d, zi_d = to_dev(e), to_dev(a), to_dev(g), to_dev(zi)
    s, zf, saved = plan.forward_ti(e_d, a_d, zi_d, want_zf=True)
    ge, ga, gz = plan.backward_ti(g_d, a_d, e_d, saved, s=s if store_s else None, zi=zi_d, need_zi=with_zi)
    plan.check_status()
    torch.cuda.synchronize()
    assert per_seq_err(host(s), s_ref) <= TOL
    assert rms_rel(host(zf), zf_ref) <= TOL
    assert per_seq_err(host(ge), ge_ref) <= TOL
    for b in range(B):
        assert rms_rel(host(ga)[b], ga_ref[b]) <= TOL, b
    if with_zi:
        assert rms_rel(host(gz), gz_ref) <= TOL


def test_time_invariant_training_shape(tv):
    """B=64, T=48000, M=22 with one coefficient row per sequence, recompute adjoint;
    every sequence against the oracle."""
    B, T, M = 64, 48000, 22
    e, a, g = _ti_inputs(B, T, M, seed=4242)
    plan = tv.Plan(M, dev())
    e_d, a_d, g_d = to_dev(e), to_dev(a), to_dev(g)
    s, _, saved = plan.forward_ti(e_d, a_d)
    ge, ga, _ = plan.backward_ti(g_d, a_d, e_d, saved)
    plan.check_status()
    torch.cuda.synchronize()
    s_ref, _ = oracle.lp_forward_ti(e, a)
    ge_ref, ga_ref, _ = oracle.lp_backward_ti(g, a, s_ref)
    assert per_seq_err(host(s), s_ref) <= TOL
    assert per_seq_err(host(ge), ge_ref) <= TOL
    assert per_seq_err(host(ga), ga_ref) <= TOL


def _framewise_inputs(B, T, M, hop, seed):
    from tests.pins import stable_ti_coeffs
    rng = np.random.default_rng(seed)
    F = oracle.framewise_geometry(T, hop)[1]
    af = np.stack([np.stack([stable_ti_coeffs(rng, M) for _ in range(F)]) for _ in range(B)]).astype(np.float32)
    return make_excitation(rng, B, T), af, make_upstream_grad(rng, B, T)


def test_frames_gather_and_overlap_add(tv):
    """The framing kernels against their definition (NumPy), weighted and not."""
    from paper_2406_05128_amd import _lib
    B, T, hop = 2, 1000, 50
    W, F = oracle.framewise_geometry(T, hop)
    assert tv.frames_count(T, hop) == F
    x = np.random.default_rng(3).standard_normal((B, T)).astype(np.float32)
    xf_d = torch.empty((B, F, W), dtype=torch.float32, device=dev())
    x_d = to_dev(x)
    w = 0.5 * oracle.hann_periodic(W)
    ref = np.zeros((B, F, W))
    for f in range(F):
        for n in range(W):
            t = (f - 3) * hop + n
            if 0 <= t < T:
                ref[:, f, n] = x[:, t]
    lib, st = _lib.load(), torch.cuda.current_stream(dev()).cuda_stream
    import ctypes
    for weighted in (0, 1):
        assert lib.lp_frames_gather(B, T, hop, ctypes.c_void_p(x_d.data_ptr()), ctypes.c_void_p(xf_d.data_ptr()),
                                    weighted, ctypes.c_void_p(st)) == 0
        torch.cuda.synchronize()
        exp = ref * (w if weighted else 1.0)
        assert np.max(np.abs(host(xf_d) - exp)) <= 1e-6
        back = torch.empty_like(x_d)
        assert lib.lp_frames_overlap_add(B, T, hop, ctypes.c_void_p(xf_d.data_ptr()), ctypes.c_void_p(back.data_ptr()),
                                         weighted, ctypes.c_void_p(st)) == 0
        torch.cuda.synchronize()
        ola = np.zeros((B, T))
        got = host(xf_d)
        for f in range(F):
            for n in range(W):
                t = (f - 3) * hop + n
                if 0 <= t < T:
                    ola[:, t] += got[:, f, n] * (w[n] if weighted else 1.0)
        assert np.max(np.abs(host(back) - ola)) <= 1e-5


@pytest.mark.parametrize("B,T,M,hop,L", [(2, 1300, 6, 60, 240), (3, 5000, 22, 240, 968), (2, 2000, 22, 240, 264)])
def test_framewise_matches_oracle(tv, B, T, M, hop, L):
    """Frame-wise approximation (frames filtered with their own rows, overlap-added):
    s, dL/de and dL/daf against the oracle."""
    e, af, g = _framewise_inputs(B, T, M, hop, seed=T + M)
    s_ref, sf_ref = oracle.framewise_forward(e, af, hop)
    ge_ref, gaf_ref = oracle.framewise_backward(g, af, sf_ref, hop)
    plan = tv.Plan(M, dev(), L)
    e_d, af_d, g_d = to_dev(e), to_dev(af), to_dev(g)
    s, ctx = tv.framewise_forward(plan, e_d, af_d, hop)
    ge, gaf = tv.framewise_backward(plan, g_d, af_d, ctx, hop)
    plan.check_status()
    torch.cuda.synchronize()
    assert per_seq_err(host(s), s_ref) <= TOL
    assert per_seq_err(host(ge), ge_ref) <= TOL
    assert per_seq_err(host(gaf), gaf_ref) <= TOL


def test_framewise_training_shape(tv):
    """Frame-wise at B=64, T=48000, M=22, hop 240 (10 ms at 24 kHz): every sequence."""
    B, T, M, hop = 64, 48000, 22, 240
    e, af, g = _framewise_inputs(B, T, M, hop, seed=99)
    plan = tv.Plan(M, dev(), 968)
    e_d, af_d, g_d = to_dev(e), to_dev(af), to_dev(g)
    s, ctx = tv.framewise_forward(plan, e_d, af_d, hop)
    ge, gaf = tv.framewise_backward(plan, g_d, af_d, ctx, hop)
    plan.check_status()
    torch.cuda.synchronize()
    s_ref, sf_ref = oracle.framewise_forward(e, af, hop)
    ge_ref, gaf_ref = oracle.framewise_backward(g, af, sf_ref, hop)
    assert per_seq_err(host(s), s_ref) <= TOL
    assert per_seq_err(host(ge), ge_ref) <= TOL
    assert per_seq_err(host(gaf), gaf_ref) <= TOL


# ---------------------------------------------------------------- frame-rate coefficients

def _frame_inputs(B, T, M, hop, seed, kappa=0.9, gamma=0.98, sigma=0.01):
    """Frame-rate LPCs from a bounded random walk of reflection coefficients (step
    N(0, sigma^2) per frame, |k| <= kappa), step-up at the frame rate and
    bandwidth expansion, plus excitation and upstream gradient.  Interpolating
    LPCs (unlike reflection coefficients) can leave the stable region between
    unrelated frames; neighbouring frames this close keep every interpolated row
    inside radius ~gamma."""
    from synth.inputs import reflection_to_lpc
    rng = np.random.default_rng(seed)
    F = oracle.coef_frames_count(T, hop)
    k = np.empty((B, F, M))
    k[:, 0] = rng.uniform(-kappa, kappa, size=(B, M))
    steps = rng.normal(0.0, sigma, size=(B, F, M))
    for f in range(1, F):
        k[:, f] = np.clip(k[:, f - 1] + steps[:, f], -kappa, kappa)
    A = (reflection_to_lpc(k) * gamma ** np.arange(1, M + 1)).astype(np.float32)
    e = make_excitation(rng, B, T)
    g = make_upstream_grad(rng, B, T)
    return e, A, g


@pytest.mark.parametrize("B,T,M,L,hop,with_zi,store_s,chained", [
    (3, 5000, 22, 418, 240, False, False, False),
    (2, 3001, 16, 256, 100, True, True, False),
    (2, 2000, 22, 264, 37, False, False, True),
    (4, 1500, 8, 96, 240, False, False, False),
    (1, 777, 32, 128, 50, True, False, False),
    (2, 4000, 6, 60, 16, False, True, False),
    (3, 999, 1, 64, 10, False, False, False),
    (2, 200, 22, 418, 240, False, False, False),
    (2, 1, 12, 48, 240, False, False, False),
])
def test_frame_rate_coefficients_match_oracle(tv, B, T, M, L, hop, with_zi, store_s, chained):
    """Frame-rate rows A [B,F,M] interpolated inside the kernels: s, grad_e,
    grad_A [B,F,M] and grad_zi against the oracle (upsampling, per-sample filter,
    adjoint of the upsampling), over several chunks per frame and frames per chunk,
    ragged and short sequences."""
    e, A, g = _frame_inputs(B, T, M, hop, seed=T + M + hop)
    zi = np.random.default_rng(9).standard_normal((B, M)) if with_zi else None
    s_ref, zf_ref = oracle.lp_forward_frames(e, A, hop, zi)
    ge_ref, gA_ref, gz_ref = oracle.lp_backward_frames(g, A, s_ref, hop, zi, need_grad_zi=with_zi)
    plan = tv.Plan(M, dev(), L, chained=chained)
    e_d, A_d, g_d, zi_d = to_dev(e), to_dev(A), to_dev(g), to_dev(zi)
    s, zf, saved = plan.forward_frames(e_d, A_d, hop, zi_d, want_zf=True)
    ge, gA, gz = plan.backward_frames(g_d, A_d, hop, e_d, saved, s=s if store_s else None, zi=zi_d,
                                      need_zi=with_zi)
    plan.check_status()
    torch.cuda.synchronize()
    errs = {"s": per_seq_err(host(s), s_ref), "zf": rms_rel(host(zf), zf_ref), "grad_e": per_seq_err(host(ge), ge_ref),
            "grad_A": max(rms_rel(host(gA)[b], gA_ref[b]) for b in range(B))}
    if with_zi:
        errs["grad_zi"] = rms_rel(host(gz), gz_ref)
    print("frame-rate", (B, T, M, L, hop), {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_frame_rate_matches_per_sample_rows(tv):
    """The in-kernel interpolation against the per-sample path fed with the same
    rows upsampled on the host: equal up to the interpolation's float32 rounding."""
    B, T, M, hop = 4, 6000, 22, 240
    e, A, g = _frame_inputs(B, T, M, hop, seed=77)
    a = oracle.upsample_frames(A, T, hop).astype(np.float32)
    plan = tv.Plan(M, dev(), 418)
    e_d, A_d, a_d, g_d = to_dev(e), to_dev(A), to_dev(a), to_dev(g)
    s_f, _, saved_f = plan.forward_frames(e_d, A_d, hop)
    ge_f, _, _ = plan.backward_frames(g_d, A_d, hop, e_d, saved_f)
    s_p, _, saved_p = plan.forward(e_d, a_d)
    ge_p, _, _ = plan.backward(g_d, a_d, e_d, saved_p, need_a=False)
    plan.check_status()
    torch.cuda.synchronize()
    assert per_seq_err(host(s_f), host(s_p).astype(np.float64)) <= 1e-5
    assert per_seq_err(host(ge_f), host(ge_p).astype(np.float64)) <= 1e-5


def test_frame_rate_training_shape(tv):
    """B=64, T=48000, M=22, hop 240 (one frame per 10 ms at 24 kHz), recompute
    adjoint at the default chunk length; every sequence against the oracle."""
    B, T, M, hop = 64, 48000, 22, 240
    e, A, g = _frame_inputs(B, T, M, hop, seed=2406, kappa=0.95)
    plan = tv.Plan(M, dev())
    e_d, A_d, g_d = to_dev(e), to_dev(A), to_dev(g)
    s, _, saved = plan.forward_frames(e_d, A_d, hop)
    ge, gA, _ = plan.backward_frames(g_d, A_d, hop, e_d, saved)
    plan.check_status()
    torch.cuda.synchronize()
    s_ref, _ = oracle.lp_forward_frames(e, A, hop)
    ge_ref, gA_ref, _ = oracle.lp_backward_frames(g, A, s_ref, hop)
    assert per_seq_err(host(s), s_ref) <= TOL
    assert per_seq_err(host(ge), ge_ref) <= TOL
    assert per_seq_err(host(gA), gA_ref) <= TOL


def test_frame_rate_rejects_hop_too_short_for_lds(tv):
    """hop 1 at chunk length 418 would stage 420 frame rows per chunk: rejected by
    the host before any launch."""
    B, T, M = 1, 1000, 22
    plan = tv.Plan(M, dev(), 418)
    e = torch.zeros((B, T), dtype=torch.float32, device=dev())
    A = torch.zeros((B, tv.coef_frames_count(T, 1), M), dtype=torch.float32, device=dev())
    with pytest.raises(Exception, match="hop"):
        plan.forward_frames(e, A, 1)
    # argument checks of the C ABI: hop outside [1, 2^20], wrong frame count
    from paper_2406_05128_amd import _lib
    import ctypes
    lib = _lib.load()
    P = ctypes.c_void_p(e.data_ptr())
    assert lib.lp_forward_frames(plan._h, B, T, 0, P, P, None, P, None, None, None) == -1
    assert lib.lp_forward_frames(plan._h, B, T, (1 << 20) + 1, P, P, None, P, None, None, None) == -1
    assert lib.lp_coef_frames_count(T, 0) == 0
    with pytest.raises(ValueError):
        plan.forward_frames(e, A[:, :-1].contiguous(), 1)


# ---------------------------------------------------------------- source-filter synthesiser

def _sf_inputs(B, T, M, hop, K, K2, seed):
    from synth import pulse_train
    rng = np.random.default_rng(seed)
    e, A, _ = _frame_inputs(B, T, M, hop, seed=seed + 1)
    F = oracle.coef_frames_count(T, hop)
    p = pulse_train(rng, B, T)
    n = make_excitation(rng, B, T)
    C = (rng.standard_normal((B, F, K)) / np.sqrt(K)).astype(np.float32)
    gain = rng.uniform(0.5, 1.5, size=(B, F)).astype(np.float32)
    h = (rng.standard_normal(K2) / np.sqrt(K2)).astype(np.float32)
    gy = make_upstream_grad(rng, B, T)
    return p, n, C, gain, A, h, gy


def test_sf_source_and_output_fir(tv):
    """The synthesiser's source kernel (frame-wise FIR noise filter, pulse train,
    interpolated gain) and the output FIR with its adjoint, against the oracle."""
    from paper_2406_05128_amd import _lib
    B, T, hop, K, K2 = 3, 2500, 70, 45, 19
    p, n, C, gain, A, h, gy = _sf_inputs(B, T, 4, hop, K, K2, seed=5)
    lib, st = _lib.load(), torch.cuda.current_stream(dev()).cuda_stream
    import ctypes
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    p_d, n_d, C_d, g_d, h_d, gy_d = map(to_dev, (p, n, C, gain, h, gy))
    u_d, x_d, y_d = (torch.empty_like(p_d) for _ in range(3))
    assert lib.lp_sf_source(B, T, hop, K, P(p_d), P(n_d), P(C_d), P(g_d), P(u_d), P(x_d), ctypes.c_void_p(st)) == 0
    assert lib.lp_fir(B, T, K2, P(x_d), P(h_d), P(y_d), ctypes.c_void_p(st)) == 0
    gs_d, gh_d = torch.empty_like(gy_d), torch.empty_like(h_d)
    work = torch.empty(lib.lp_fir_adjoint_work_bytes(B, T, K2), dtype=torch.uint8, device=dev())
    assert lib.lp_fir_adjoint(B, T, K2, P(gy_d), P(x_d), P(h_d), P(gs_d), P(gh_d), P(work), ctypes.c_void_p(st)) == 0
    torch.cuda.synchronize()
    u_ref = p + oracle.framewise_fir(n, C, hop)
    gam = oracle.upsample_frames(gain[..., None].astype(np.float64), T, hop)[..., 0]
    x_ref = gam * u_ref
    assert per_seq_err(host(u_d), u_ref) <= 1e-6
    assert per_seq_err(host(x_d), x_ref) <= 1e-6
    x32 = host(x_d)
    assert per_seq_err(host(y_d), oracle.fir(x32, h)) <= 1e-6
    gs_ref, gh_ref = oracle.fir_adjoint(gy, x32, h)
    assert per_seq_err(host(gs_d), gs_ref) <= 1e-6
    assert rms_rel(host(gh_d), gh_ref) <= 1e-6


@pytest.mark.parametrize("B,T,M,hop,K,K2,L", [
    (2, 3000, 16, 100, 33, 17, 256),
    (2, 4801, 22, 240, 510, 128, 418),
    (1, 500, 8, 37, 64, 5, 96),
    (2, 1000, 22, 240, 1024, 128, 264),
    (3, 777, 12, 16, 7, 1, 48),
])
def test_sf_synth_matches_oracle(tv, B, T, M, hop, K, K2, L):
    """The whole synthesiser step (source, frame-rate LP, output FIR) and its
    adjoint through the C ABI against the oracle: y and the gradients of the
    pulse train, the noise-filter taps, the gains, the LP frame rows and the
    output FIR."""
    p, n, C, gain, A, h, gy = _sf_inputs(B, T, M, hop, K, K2, seed=T + K)
    y_ref, inter = oracle.sf_forward(p, n, C, gain, A, h, hop)
    gp_ref, gC_ref, gg_ref, gA_ref, gh_ref = oracle.sf_backward(gy, n, C, gain, A, h, inter, hop)
    syn = tv.SFSynth(M, hop, K, K2, dev(), chunk=L)
    y, ctx = syn.forward(*map(to_dev, (p, n, C, gain, A, h)))
    gp, gC, gg, gA, gh = syn.backward(to_dev(gy), ctx)
    syn.plan.check_status()
    torch.cuda.synchronize()
    errs = {"y": per_seq_err(host(y), y_ref), "grad_p": per_seq_err(host(gp), gp_ref),
            "grad_C": max(rms_rel(host(gC)[b], gC_ref[b]) for b in range(B)),
            "grad_gain": max(rms_rel(host(gg)[b], gg_ref[b]) for b in range(B)),
            "grad_A": max(rms_rel(host(gA)[b], gA_ref[b]) for b in range(B)),
            "grad_h": rms_rel(host(gh), gh_ref)}
    print("sf", (B, T, M, hop, K, K2, L), {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_sf_synth_training_shape(tv):
    """B=64, T=48000, M=22, hop 240, a 510-tap noise filter per frame (256
    frequency bins) and a 128-tap output FIR: every output and gradient against
    the oracle on the whole batch."""
    B, T, M, hop, K, K2 = 64, 48000, 22, 240, 510, 128
    p, n, C, gain, A, h, gy = _sf_inputs(B, T, M, hop, K, K2, seed=2024)
    syn = tv.SFSynth(M, hop, K, K2, dev())
    y, ctx = syn.forward(*map(to_dev, (p, n, C, gain, A, h)))
    gp, gC, gg, gA, gh = syn.backward(to_dev(gy), ctx)
    syn.plan.check_status()
    torch.cuda.synchronize()
    y_ref, inter = oracle.sf_forward(p, n, C, gain, A, h, hop)
    gp_ref, gC_ref, gg_ref, gA_ref, gh_ref = oracle.sf_backward(gy, n, C, gain, A, h, inter, hop)
    assert per_seq_err(host(y), y_ref) <= TOL
    assert per_seq_err(host(gp), gp_ref) <= TOL
    assert per_seq_err(host(gC), gC_ref) <= TOL
    assert per_seq_err(host(gg), gg_ref) <= TOL
    assert per_seq_err(host(gA), gA_ref) <= TOL
    assert rms_rel(host(gh), gh_ref) <= TOL


def test_sf_rejects_out_of_range_sizes(tv):
    """FIR longer than 1024 taps and frames longer than 4096 samples are refused."""
    from paper_2406_05128_amd import _lib
    lib = _lib.load()
    z = torch.zeros(16, dtype=torch.float32, device=dev())
    import ctypes
    P = ctypes.c_void_p(z.data_ptr())
    assert lib.lp_fir(1, 4, 1025, P, P, P, None) == -1
    assert b"K" in lib.lp_sf_last_error()
    assert lib.lp_sf_source(1, 4, 5000, 2, P, P, P, P, P, P, None) == -1


def test_autograd_frame_rate_and_synthesiser(tv):
    """torch.autograd wrappers: lp_frames (grads of e, A and zi) and sf_synth (grads
    of p, C, gain, A, h) against the oracle."""
    B, T, M, hop = 2, 2500, 16, 120
    e, A, g = _frame_inputs(B, T, M, hop, seed=88)
    zi = np.random.default_rng(3).standard_normal((B, M))
    e_d = to_dev(e).requires_grad_(True)
    A_d = to_dev(A).requires_grad_(True)
    zi_d = to_dev(zi).requires_grad_(True)
    s = tv.lp_frames(e_d, A_d, hop, zi_d, chunk=160)
    s.backward(to_dev(g))
    torch.cuda.synchronize()
    s_ref, _ = oracle.lp_forward_frames(e, A, hop, zi)
    ge_ref, gA_ref, gz_ref = oracle.lp_backward_frames(g, A, s_ref, hop, zi, need_grad_zi=True)
    assert per_seq_err(host(s), s_ref) <= TOL
    assert per_seq_err(host(e_d.grad), ge_ref) <= TOL
    assert max(rms_rel(host(A_d.grad)[b], gA_ref[b]) for b in range(B)) <= TOL
    assert rms_rel(host(zi_d.grad), gz_ref) <= TOL

    K, K2 = 40, 9
    p, n, C, gain, A, h, gy = _sf_inputs(B, T, M, hop, K, K2, seed=89)
    leaves = [to_dev(x).requires_grad_(True) for x in (p, C, gain, A, h)]
    p_d, C_d, g_d, A_d, h_d = leaves
    y = tv.sf_synth(p_d, to_dev(n), C_d, g_d, A_d, h_d, hop)
    y.backward(to_dev(gy))
    torch.cuda.synchronize()
    y_ref, inter = oracle.sf_forward(p, n, C, gain, A, h, hop)
    refs = oracle.sf_backward(gy, n, C, gain, A, h, inter, hop)
    assert per_seq_err(host(y), y_ref) <= TOL
    for leaf, ref, name in zip(leaves, refs, ("p", "C", "gain", "A", "h")):
        got = host(leaf.grad)
        err = rms_rel(got, ref) if name == "h" else max(rms_rel(got[b], ref[b]) for b in range(B))
        assert err <= TOL, (name, err)


def test_frame_rate_hop1_equals_per_sample_rows(tv):
    """hop 1: every sample is a frame sample, so the frame-rate path must give the
    per-sample path's results for rows A[:, :T] (and a zero gradient for the extra
    row), through different kernel instantiations."""
    B, T, M, hop, L = 2, 3000, 22, 1, 44
    e, A, g = _frame_inputs(B, T, M, hop, seed=12)
    plan = tv.Plan(M, dev(), L)
    e_d, A_d, g_d = to_dev(e), to_dev(A), to_dev(g)
    a_d = A_d[:, :T].contiguous()
    s_f, _, sv_f = plan.forward_frames(e_d, A_d, hop)
    ge_f, gA_f, _ = plan.backward_frames(g_d, A_d, hop, e_d, sv_f)
    s_p, _, sv_p = plan.forward(e_d, a_d)
    ge_p, ga_p, _ = plan.backward(g_d, a_d, e_d, sv_p)
    plan.check_status()
    torch.cuda.synchronize()
    assert per_seq_err(host(s_f), host(s_p).astype(np.float64)) <= 1e-6
    assert per_seq_err(host(ge_f), host(ge_p).astype(np.float64)) <= 1e-6
    for b in range(B):
        assert rms_rel(host(gA_f)[b, :T], host(ga_p)[b].astype(np.float64)) <= 1e-5, b
    assert np.all(host(gA_f)[:, T] == 0.0)


@pytest.mark.parametrize("T", [100, 239, 241, 700])
def test_sf_synth_short_signals(tv, T):
    """The synthesiser on signals shorter than a frame (hop 240) and than the noise
    filter (510 taps), against the oracle."""
    B, M, hop, K, K2 = 2, 22, 240, 510, 128
    p, n, C, gain, A, h, gy = _sf_inputs(B, T, M, hop, K, K2, seed=T)
    syn = tv.SFSynth(M, hop, K, K2, dev(), chunk=264)
    y, ctx = syn.forward(*map(to_dev, (p, n, C, gain, A, h)))
    gp, gC, gg, gA, gh = syn.backward(to_dev(gy), ctx)
    syn.plan.check_status()
    torch.cuda.synchronize()
    y_ref, inter = oracle.sf_forward(p, n, C, gain, A, h, hop)
    refs = oracle.sf_backward(gy, n, C, gain, A, h, inter, hop)
    assert per_seq_err(host(y), y_ref) <= TOL
    for got, ref, name in zip((gp, gC, gg, gA, gh), refs, ("p", "C", "gain", "A", "h")):
        got = host(got)
        err = rms_rel(got, ref) if name == "h" else max(rms_rel(got[b], ref[b]) for b in range(B))
        assert err <= TOL, (name, err)
