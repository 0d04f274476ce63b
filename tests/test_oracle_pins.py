"""The float64 oracle against what the paper and mathematics fix (CPU only)."""
import numpy as np
import pytest

import oracle
from tests import pins


@pytest.fixture(scope="module", autouse=True)
def _built_oracle():
    oracle.build(force=False)


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin(oracle.lp_forward, oracle.lp_backward)


# --------------------------------------------------------------------------
# Planted mistakes: each plausible error in the oracle must fail some pin.
# The mistakes are planted by wrapping the CPU oracle, never on a GPU.

def _fwd_coef_time_shift(e, a, zi=None):
    # uses a(t-1) for output t instead of a(t)
    a2 = np.array(a, np.float64, copy=True)
    a2[:, 1:] = a2[:, :-1].copy()
    return oracle.lp_forward(e, a2, zi)


def _fwd_dropped_last_tap(e, a, zi=None):
    a2 = np.array(a, np.float64, copy=True)
    a2[..., -1] = 0.0
    return oracle.lp_forward(e, a2, zi)


def _fwd_sign_flip(e, a, zi=None):
    a2 = -np.array(a, np.float64)
    z2 = None if zi is None else np.asarray(zi)
    return oracle.lp_forward(e, a2, z2)


def _fwd_reversed_taps(e, a, zi=None):
    # a_i paired with s(t-(M+1-i)) — a transposed operand
    return oracle.lp_forward(e, np.array(a, np.float64)[..., ::-1].copy(), zi)


def _bwd_unshifted(g, a, s, zi=None, need_grad_a=True, need_grad_zi=False):
    # adjoint that forgets the shift ahat_i(t) = a_i(t+i) and uses a_i(t)
    a64 = np.array(a, np.float64)
    ghat = oracle.lp_forward(np.array(g, np.float64)[:, ::-1].copy(), a64[:, ::-1].copy())[0][:, ::-1]
    ge = ghat.copy()
    B, T, M = a64.shape
    ga = np.zeros((B, T, M))
    for i in range(1, M + 1):
        ga[:, i:, i - 1] = -ge[:, i:] * s[:, :-i] if i < T else 0.0
    return ge, ga, (np.zeros((B, M)) if need_grad_zi else None)


def _bwd_wrong_lag(g, a, s, zi=None, need_grad_a=True, need_grad_zi=False):
    ge, ga, gz = oracle.lp_backward(g, a, s, zi, True, need_grad_zi)
    B, T, M = ga.shape
    ga2 = np.zeros_like(ga)
    for i in range(1, M + 1):  # pairs ghat(t) with s(t-i+1)
        ga2[:, i - 1:, i - 1] = -ge[:, i - 1:] * s[:, :T - i + 1]
    return ge, ga2, gz


def _bwd_grad_a_sign(g, a, s, zi=None, need_grad_a=True, need_grad_zi=False):
    ge, ga, gz = oracle.lp_backward(g, a, s, zi, True, need_grad_zi)
    return ge, -ga, gz


MUTANTS = {
    "coef_time_shift": (_fwd_coef_time_shift, oracle.lp_backward),
    "dropped_last_tap": (_fwd_dropped_last_tap, oracle.lp_backward),
    "sign_flip": (_fwd_sign_flip, oracle.lp_backward),
    "reversed_taps": (_fwd_reversed_taps, oracle.lp_backward),
    "bwd_unshifted": (oracle.lp_forward, _bwd_unshifted),
    "grad_a_wrong_lag": (oracle.lp_forward, _bwd_wrong_lag),
    "grad_a_sign": (oracle.lp_forward, _bwd_grad_a_sign),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    fwd, bwd = MUTANTS[name]
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(fwd, bwd)
        except (AssertionError, ValueError, IndexError, FloatingPointError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"


def test_oracle_time_invariant_entry_points():
    """lp_forward_ti / lp_backward_ti against scipy.signal.lfilter (Eq. 2) and the
    time-invariant coefficient gradient of Eq. 4, with a nonzero initial state."""
    import scipy.signal
    rng = np.random.default_rng(31)
    B, T, M = 2, 400, 6
    a = np.stack([pins.stable_ti_coeffs(rng, M) for _ in range(B)])
    e = rng.standard_normal((B, T)); g = rng.standard_normal((B, T))
    zi = rng.standard_normal((B, M))
    s, zf = oracle.lp_forward_ti(e, a, zi)
    ge, ga, gz = oracle.lp_backward_ti(g, a, s, zi, need_grad_zi=True)
    for b in range(B):
        den = np.concatenate([[1.0], a[b]])
        # the initial state s(-1..-M) = zi expressed as lfilter's direct-form-II-transposed state
        zi_lf = scipy.signal.lfiltic([1.0], den, y=zi[b])
        ref_s, _ = scipy.signal.lfilter([1.0], den, e[b], zi=zi_lf)
        assert pins.rms_rel(s[b], ref_s) < 1e-12
        assert pins.rms_rel(zf[b], s[b, ::-1][:M]) < 1e-15
        # Eq. 4: dL/da_i = sum_t g(t) LP_a(-s(t-i)), the history before t = 0 being zi
        ext = np.concatenate([zi[b][::-1], s[b]])  # ext[M + t] = s(t), ext[M - 1 - k] = s(-1-k)
        for i in range(1, M + 1):
            shifted = -ext[M - i:M - i + T]
            ref = float(np.dot(g[b], scipy.signal.lfilter([1.0], den, shifted)))
            assert abs(float(ga[b, i - 1]) - ref) <= 1e-10 * (abs(ref) + 1.0), (b, i)
    # dL/dzi by central differences of L = <g, s>
    h = 1e-6
    for j in range(M):
        zp = zi.copy(); zp[0, j] += h
        zm = zi.copy(); zm[0, j] -= h
        fd = (np.dot(g[0], oracle.lp_forward_ti(e, a, zp)[0][0]) - np.dot(g[0], oracle.lp_forward_ti(e, a, zm)[0][0])) / (2 * h)
        assert abs(fd - gz[0, j]) <= 1e-6 * (abs(fd) + 1.0)


def test_oracle_framewise_approximation():
    """Frame-wise approximation (time-invariant filter per frame, Hann overlap-add at
    75 % overlap): an independent per-frame scipy.signal.lfilter computation, the
    identity filter reconstructing its input, the adjoint identity in e, and
    central finite differences for the frame coefficients."""
    import scipy.signal
    rng = np.random.default_rng(41)
    B, T, M, hop = 2, 1300, 5, 60
    W, F = oracle.framewise_geometry(T, hop)
    af = np.stack([np.stack([pins.stable_ti_coeffs(rng, M) for _ in range(F)]) for _ in range(B)])
    e = rng.standard_normal((B, T)); g = rng.standard_normal((B, T))
    s, sf = oracle.framewise_forward(e, af, hop)
    # independent: lfilter on each frame, window, overlap-add, halve
    w = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(W) / W)
    ref = np.zeros((B, T))
    for b in range(B):
        padded = np.concatenate([np.zeros(3 * hop), e[b], np.zeros(W)])
        out = np.zeros(T + 3 * hop + W)
        for f in range(F):
            y = scipy.signal.lfilter([1.0], np.concatenate([[1.0], af[b, f]]), padded[f * hop:f * hop + W])
            out[f * hop:f * hop + W] += w * y
        ref[b] = 0.5 * out[3 * hop:3 * hop + T]
    assert pins.rms_rel(s, ref) < 1e-12
    # identity filter: the windows sum to 2, so the output is the input
    s0, sf0 = oracle.framewise_forward(e, np.zeros_like(af), hop)
    assert np.max(np.abs(s0 - e)) < 1e-12
    ge0, _ = oracle.framewise_backward(g, np.zeros_like(af), sf0, hop)
    assert np.max(np.abs(ge0 - g)) < 1e-12
    # adjoint identity in e: <g, FW(x)> = <FW^T(g), x>
    ge, gaf = oracle.framewise_backward(g, af, sf, hop)
    x = rng.standard_normal((B, T))
    lhs = float(np.sum(g * oracle.framewise_forward(x, af, hop)[0]))
    rhs = float(np.sum(oracle.framewise_backward(g, af, oracle.framewise_forward(x, af, hop)[1], hop)[0] * x))
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1.0)
    # finite differences of L = <g, s> for a few frame coefficients
    h = 1e-6
    for (b, f, i) in [(0, 3, 0), (1, 10, 4), (0, F - 1, 2), (1, 0, 1)]:
        ap = af.copy(); ap[b, f, i] += h
        am = af.copy(); am[b, f, i] -= h
        fd = (np.sum(g * oracle.framewise_forward(e, ap, hop)[0]) - np.sum(g * oracle.framewise_forward(e, am, hop)[0])) / (2 * h)
        assert abs(fd - gaf[b, f, i]) <= 1e-6 * (abs(fd) + 1.0), (b, f, i, fd, gaf[b, f, i])


def test_oracle_frame_rate_coefficients():
    """Frame-rate LP coefficients linearly upsampled to the sample rate (Sec. 4.3):
    the upsampling against numpy.interp and its values at the frame samples, a
    constant track against the time-invariant filter, hop 1 against the
    per-sample adjoint, the adjoint identity of the upsampling, and central
    finite differences of L = <g, s> in the frame coefficients."""
    from synth.inputs import reflection_to_lpc
    rng = np.random.default_rng(43)
    B, T, M, hop = 2, 700, 6, 50
    F = oracle.coef_frames_count(T, hop)
    assert F == 15
    A = reflection_to_lpc(rng.uniform(-0.7, 0.7, size=(B, F, M)))
    a = oracle.upsample_frames(A, T, hop)
    # numpy.interp between frame samples q*hop, coefficient by coefficient
    xp = np.arange(F) * hop
    for b in range(B):
        for i in range(M):
            ref = np.interp(np.arange(T), xp, A[b, :, i])
            assert np.max(np.abs(a[b, :, i] - ref)) <= 1e-14 * (1.0 + np.max(np.abs(ref)))
    # the frame samples carry the frame rows exactly
    qs = np.arange(0, T, hop)
    assert np.array_equal(a[:, qs, :], A[:, qs // hop, :])
    e = rng.standard_normal((B, T)); g = rng.standard_normal((B, T))
    # a constant track is the time-invariant filter
    Ac = np.repeat(A[:, :1, :], F, axis=1).astype(np.float32)
    s_c, _ = oracle.lp_forward_frames(e, Ac, hop)
    s_ti, _ = oracle.lp_forward_ti(e, Ac[:, 0, :])
    assert pins.rms_rel(s_c, s_ti) < 1e-12
    # hop 1: every sample has its own row; the frame gradient is the per-sample one
    A1 = reflection_to_lpc(rng.uniform(-0.5, 0.5, size=(B, T + 1, M))).astype(np.float32)
    s1, _ = oracle.lp_forward_frames(e, A1, 1)
    ge1, gA1, _ = oracle.lp_backward_frames(g, A1, s1, 1)
    ge_ref, ga_ref, _ = oracle.lp_backward(g, A1[:, :T], s1)
    assert np.array_equal(ge1, ge_ref)
    assert np.allclose(gA1[:, :T], ga_ref, rtol=0, atol=1e-12 * np.max(np.abs(ga_ref)))
    assert np.all(gA1[:, T] == 0.0)
    # adjoint identity of the upsampling: <up(X), Y> = <X, up^T(Y)>
    X = rng.standard_normal((B, F, M)); Y = rng.standard_normal((B, T, M))
    lhs = float(np.sum(oracle.upsample_frames(X, T, hop) * Y))
    rhs = float(np.sum(X * oracle.upsample_frames_adjoint(Y, F, hop)))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1.0)
    # finite differences of L = <g, s> in the frame coefficients (float64 rows)
    s, _ = oracle.lp_forward_frames(e, A, hop, round_rows=False)
    ge, gA, _ = oracle.lp_backward_frames(g, A, s, hop, round_rows=False)
    h = 1e-6
    for (b, q, i) in [(0, 0, 0), (1, 4, 3), (0, F - 1, 5), (1, F - 2, 1), (0, 7, 2)]:
        ap = A.copy(); ap[b, q, i] += h
        am = A.copy(); am[b, q, i] -= h
        fd = (np.sum(g * oracle.lp_forward_frames(e, ap, hop, round_rows=False)[0])
              - np.sum(g * oracle.lp_forward_frames(e, am, hop, round_rows=False)[0])) / (2 * h)
        assert abs(fd - gA[b, q, i]) <= 1e-6 * (abs(fd) + 1.0), (b, q, i, fd, gA[b, q, i])
    # the excitation gradient is the per-sample one on the upsampled rows
    ge_ps, _, _ = oracle.lp_backward(g, a, s)
    assert np.array_equal(ge, ge_ps)
    # by default the filter reads the rows rounded once to float32
    s_r, _ = oracle.lp_forward_frames(e, A, hop)
    assert np.array_equal(s_r, oracle.lp_forward(e, a.astype(np.float32))[0])


def test_frame_row_rounding_effect_on_record():
    """How far the float32 rounding of the upsampled rows (the reading of Sec. 4.3
    that the upsampled coefficients are float32 tensors) moves the filter against
    float64 rows, at the frame-rate training shape (T = 48000, M = 22, hop 240,
    random-walk reflection coefficients |k| <= 0.95, bandwidth 0.98) on 4
    sequences.  Each rounded row differs from its float64 value by at most half a
    float32 ulp, and the filter amplifies that by its conditioning: the median
    moves by about 1e-6 rms-relative, the most resonant sequences by up to a few
    1e-4 (the full 64-sequence batch: s 2.8e-4, grad_e 2.8e-4, grad_A 4.2e-4)."""
    from synth.inputs import reflection_to_lpc
    rng = np.random.default_rng(78)
    B, T, M, hop = 4, 48000, 22, 240
    F = oracle.coef_frames_count(T, hop)
    k = np.empty((B, F, M))
    k[:, 0] = rng.uniform(-0.95, 0.95, size=(B, M))
    dk = rng.normal(0.0, 0.01, size=(B, F, M))
    for f in range(1, F):
        k[:, f] = np.clip(k[:, f - 1] + dk[:, f], -0.95, 0.95)
    A = (reflection_to_lpc(k) * 0.98 ** np.arange(1, M + 1)).astype(np.float32)
    e = rng.standard_normal((B, T)).astype(np.float32)
    g = rng.standard_normal((B, T)).astype(np.float32)
    # the rounded rows are within half an ulp of the float64 rows
    a64 = oracle.upsample_frames(A, T, hop)
    a32 = a64.astype(np.float32)
    assert np.all(np.abs(a32 - a64) <= 0.5 * np.spacing(np.abs(a32)).astype(np.float64) * (1 + 1e-12))
    res = {}
    for rr in (True, False):
        s, _ = oracle.lp_forward_frames(e, A, hop, round_rows=rr)
        ge, gA, _ = oracle.lp_backward_frames(g, A, s, hop, round_rows=rr)
        res[rr] = (s, ge, gA)
    for name, i in (("s", 0), ("grad_e", 1), ("grad_A", 2)):
        d = [pins.rms_rel(res[True][i][b], res[False][i][b]) for b in range(B)]
        print(f"float32 rows vs float64 rows, {name}: median {np.median(d):.2e} max {max(d):.2e}")
        # rounding moves every result, by far less than the results themselves
        assert 0.0 < np.median(d) < 1e-4
        assert max(d) < 1e-3


def test_oracle_source_filter_synthesiser():
    """The source-filter synthesiser of Eq. 5 around the LP filter: the frame-wise
    noise FIR against numpy.convolve (identical taps) and a per-sample double loop
    (varying taps), the output FIR against scipy.signal.lfilter, adjoint
    identities, the reduction to the LP filter alone, and central finite
    differences for every parameter gradient."""
    import scipy.signal
    from synth.inputs import reflection_to_lpc
    rng = np.random.default_rng(47)
    B, T, M, hop, K, K2 = 2, 400, 6, 50, 9, 5
    F = oracle.coef_frames_count(T, hop)
    n = rng.standard_normal((B, T)); p = rng.standard_normal((B, T))
    C = 0.3 * rng.standard_normal((B, F, K))
    # identical taps in every frame: one convolution of the whole signal
    Cs = np.repeat(C[:, :1], F, axis=1)
    u1 = oracle.framewise_fir(n, Cs, hop)
    for b in range(B):
        assert np.max(np.abs(u1[b] - np.convolve(n[b], Cs[b, 0])[:T])) < 1e-12
    # varying taps: each input sample filtered by its own frame's taps
    u2 = oracle.framewise_fir(n, C, hop)
    ref = np.zeros((B, T))
    for b in range(B):
        for t in range(T):
            for k in range(K):
                if t - k >= 0:
                    ref[b, t] += C[b, (t - k) // hop, k] * n[b, t - k]
    assert np.max(np.abs(u2 - ref)) < 1e-12
    # the output FIR is lfilter with numerator h
    h = rng.standard_normal(K2)
    s = rng.standard_normal((B, T))
    assert np.max(np.abs(oracle.fir(s, h) - scipy.signal.lfilter(h, [1.0], s, axis=1))) < 1e-12
    # adjoint identities: frame-wise FIR in its taps, output FIR in s and in h
    gy = rng.standard_normal((B, T))
    gC = oracle.framewise_fir_adjoint(gy, n, F, K, hop)
    assert abs(np.sum(gy * u2) - np.sum(gC * C)) < 1e-9 * (1 + abs(np.sum(gy * u2)))
    gs, gh = oracle.fir_adjoint(gy, s, h)
    y = oracle.fir(s, h)
    assert abs(np.sum(gy * y) - np.sum(gs * s)) < 1e-9 * (1 + abs(np.sum(gy * y)))
    assert abs(np.sum(gy * y) - np.sum(gh * h)) < 1e-9 * (1 + abs(np.sum(gy * y)))
    # the whole synthesiser
    A = (reflection_to_lpc(rng.uniform(-0.6, 0.6, size=(B, F, M))) * 0.98 ** np.arange(1, M + 1))
    gain = rng.uniform(0.5, 1.5, size=(B, F))
    # no noise, unit gain, identity output filter: the LP filter of the pulse train
    delta = np.zeros(K2); delta[0] = 1.0
    y0, _ = oracle.sf_forward(p, n, np.zeros_like(C), np.ones_like(gain), A, delta, hop)
    assert np.max(np.abs(y0 - oracle.lp_forward_frames(p, A, hop)[0])) < 1e-12
    y, inter = oracle.sf_forward(p, n, C, gain, A, h, hop, round_rows=False)
    gp, gCs, ggain, gA, ghs = oracle.sf_backward(gy, n, C, gain, A, h, inter, hop, round_rows=False)

    def loss(**kw):
        args = dict(p=p, C=C, gain=gain, A=A, h=h)
        args.update(kw)
        return float(np.sum(gy * oracle.sf_forward(args["p"], n, args["C"], args["gain"], args["A"], args["h"], hop,
                                                   round_rows=False)[0]))

    eps = 1e-6
    for name, arr, grad, idx in [("p", p, gp, (1, 123)), ("C", C, gCs, (0, 3, 4)), ("C", C, gCs, (1, 7, 0)),
                                 ("gain", gain, ggain, (0, 2)), ("gain", gain, ggain, (1, F - 1)),
                                 ("A", A, gA, (1, 5, 2)), ("h", h, ghs, (3,))]:
        ap = arr.copy(); ap[idx] += eps
        am = arr.copy(); am[idx] -= eps
        fd = (loss(**{name: ap}) - loss(**{name: am})) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * (abs(fd) + 1.0), (name, idx, fd, grad[idx])
