"""Independent checks that pin the float64 oracle to the paper and to mathematics.

Each ``check_*`` takes the forward / backward callables under test (normally
the oracle's ``lp_forward`` / ``lp_backward``) and raises AssertionError when
they disagree with something the paper or linear algebra fixes:

* closed forms of the order-1 filter (Eq. 6 with M = 1),
* the time-invariant special case against ``scipy.signal.lfilter`` (Eq. 2) and
  the paper's two-filter time-invariant gradients (Eqs. 3-4),
* a dense triangular solve of A s = e, A[t,t] = 1, A[t,t-i] = a_i(t),
* the impulse-response expansion of Eqs. 7-9, enumerated by brute force,
* linearity in e and state continuation,
* the adjoint identity <y, LP(x)> = <LP^T(y), x> and the dense A^-T g,
* float64 central finite differences for dL/de, dL/da and dL/dzi.

None of these re-types the oracle's recursion: they use a library routine, a
different formula from the paper, or a mathematical identity.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import scipy.linalg
import scipy.signal

from synth import make_coeffs, reflection_to_lpc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rms_rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.sqrt(np.mean(ref ** 2))
    return float(np.sqrt(np.mean((x - ref) ** 2)) / (den if den > 0 else 1.0))


def max_rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / (den if den > 0 else 1.0))


# --------------------------------------------------------------------------- helpers

def dense_A(a_seq: np.ndarray) -> np.ndarray:
    """Unit lower-triangular banded matrix of the filter: (A s)(t) = e(t)."""
    T, M = a_seq.shape
    A = np.eye(T)
    for t in range(T):
        for i in range(1, M + 1):
            if t - i >= 0:
                A[t, t - i] = a_seq[t, i - 1]
    return A


def compositions(d: int, M: int):
    """The set G_d of Eq. 9: ordered tuples of parts in 1..M summing to d; G_0 = {()}."""
    if d == 0:
        yield ()
        return
    for i in range(1, min(d, M) + 1):
        for q in compositions(d - i, M):
            yield (i,) + q


def b_coeff(a_seq: np.ndarray, d: int, t: int) -> float:
    """Eq. 8: b_d(t) = sum_{q in G_d} (-1)^|q| prod_j a_{q_j}(t - sum_{k<=j} Q(q)_k), Q(q) = [0; q]."""
    M = a_seq.shape[1]
    total = 0.0
    for q in compositions(d, M):
        Q = (0,) + q
        prod = 1.0
        for j in range(1, len(q) + 1):
            tau = t - sum(Q[:j])
            prod *= a_seq[tau, q[j - 1] - 1]
        total += (-1.0) ** len(q) * prod
    return total


def stable_ti_coeffs(rng, M, radius=0.95):
    k = rng.uniform(-0.9, 0.9, size=M)
    a = reflection_to_lpc(k)
    return a * radius ** np.arange(1, M + 1)


def tv_coeffs(rng, T, M, kappa=0.9, gamma=0.95):
    return make_coeffs(rng, 1, T, M, kappa, gamma).astype(np.float64)[0]


# --------------------------------------------------------------------------- forward pins

def check_golden_worked_example(fwd, bwd):
    with open(os.path.join(GOLDEN, "worked_m2_t4.json")) as f:
        gold = json.load(f)
    e = np.array(gold["e"], np.float32)[None]
    a = np.array(gold["a"], np.float32)[None]
    g = np.array(gold["g"], np.float32)[None]
    s, _ = fwd(e, a)
    assert np.array_equal(s[0], np.array(gold["s"])), (s, gold["s"])
    ge, ga, _ = bwd(g, a, s)
    assert np.array_equal(ge[0], np.array(gold["grad_e"])), (ge, gold["grad_e"])
    assert np.array_equal(ga[0], np.array(gold["grad_a"])), (ga, gold["grad_a"])


def check_m1_closed_forms(fwd, bwd):
    # time-invariant: a_1 = -rho, e = delta  ->  s(t) = rho^t
    T, rho = 60, 0.9
    e = np.zeros((1, T)); e[0, 0] = 1.0
    a = np.full((1, T, 1), -rho)
    s, _ = fwd(e, a)
    np.testing.assert_allclose(s[0], rho ** np.arange(T), rtol=1e-13, atol=0)
    # time-varying: s(t) = prod_{tau=1..t} (-a_1(tau))
    rng = np.random.default_rng(7)
    a = rng.uniform(-1.1, 1.1, size=(1, T, 1))
    s, _ = fwd(e, a)
    ref = np.concatenate([[1.0], np.cumprod(-a[0, 1:, 0])])
    np.testing.assert_allclose(s[0], ref, rtol=1e-12, atol=1e-300)


def check_ti_lfilter(fwd, bwd):
    rng = np.random.default_rng(11)
    for M in (1, 2, 6, 16):
        T = 400
        c = stable_ti_coeffs(rng, M)
        e = rng.standard_normal((1, T))
        a = np.broadcast_to(c, (1, T, M)).copy()
        s, _ = fwd(e, a)
        ref = scipy.signal.lfilter([1.0], np.concatenate([[1.0], c]), e[0])
        assert rms_rel(s[0], ref) < 1e-12, (M, rms_rel(s[0], ref))


def check_dense_forward(fwd, bwd):
    rng = np.random.default_rng(12)
    for (T, M) in ((1, 3), (5, 8), (64, 5), (300, 22)):
        a = tv_coeffs(rng, T, M)
        e = rng.standard_normal(T)
        s, _ = fwd(e[None], a[None])
        ref = scipy.linalg.solve_triangular(dense_A(a), e, lower=True, unit_diagonal=True)
        assert rms_rel(s[0], ref) < 1e-12, (T, M, rms_rel(s[0], ref))


def check_composition_expansion(fwd, bwd):
    """Eq. 7-9: impulse responses and the convolution form by brute-force enumeration."""
    rng = np.random.default_rng(13)
    for (T, M) in ((12, 1), (12, 2), (13, 3), (12, 4)):
        a = rng.uniform(-0.8, 0.8, size=(T, M))
        # columns: response at t to a unit impulse at tau equals b_{t-tau}(t)
        for tau in (0, 1, 5):
            e = np.zeros(T); e[tau] = 1.0
            s, _ = fwd(e[None], a[None])
            ref = np.zeros(T)
            for t in range(tau, T):
                ref[t] = 1.0 if t == tau else b_coeff(a, t - tau, t)
            np.testing.assert_allclose(s[0], ref, rtol=1e-12, atol=1e-12)
        # Eq. 7: s(t) = e(t) + sum_{d=1..t} b_d(t) e(t-d), for a random e
        e = rng.standard_normal(T)
        s, _ = fwd(e[None], a[None])
        conv = np.array([e[t] + sum(b_coeff(a, d, t) * e[t - d] for d in range(1, t + 1))
                         for t in range(T)])
        np.testing.assert_allclose(s[0], conv, rtol=1e-11, atol=1e-11)


def check_linearity_and_continuation(fwd, bwd):
    rng = np.random.default_rng(14)
    T, M = 500, 10
    a = tv_coeffs(rng, T, M)[None]
    x = rng.standard_normal((1, T)); y = rng.standard_normal((1, T))
    sx, _ = fwd(x, a); sy, _ = fwd(y, a)
    sxy, _ = fwd(2.5 * x - 0.75 * y, a)
    assert rms_rel(sxy, 2.5 * sx - 0.75 * sy) < 1e-12
    # continuation: run [0,T1) then [T1,T) from the carried state == one shot
    for T1 in (3, 137, 499):
        s1, zf1 = fwd(x[:, :T1], a[:, :T1])
        s2, zf2 = fwd(x[:, T1:], a[:, T1:], zf1)
        full, zf = fwd(x, a)
        assert rms_rel(np.concatenate([s1, s2], axis=1), full) < 1e-13
        np.testing.assert_allclose(zf2, zf, rtol=1e-12, atol=1e-12)


def check_state_is_past_outputs(fwd, bwd):
    """zi = [s(-1..-M)] means the same as prepending those outputs (Sec. 2.2 conventions)."""
    rng = np.random.default_rng(15)
    T, M = 40, 6
    a_full = tv_coeffs(rng, T + M, M)[None]
    e_full = rng.standard_normal((1, T + M))
    # zero-state run over a prefix of length M produces s(0..M-1); use them as zi for the rest
    s_full, _ = fwd(e_full, a_full)
    zi = s_full[:, M - 1::-1][:, :M]  # s(M-1), s(M-2), ..., s(0)
    s_tail, _ = fwd(e_full[:, M:], a_full[:, M:], zi)
    assert rms_rel(s_tail, s_full[:, M:]) < 1e-13


# --------------------------------------------------------------------------- adjoint pins

def check_adjoint_identity(fwd, bwd):
    rng = np.random.default_rng(21)
    for (T, M) in ((1, 4), (7, 3), (800, 16), (600, 22)):
        a = tv_coeffs(rng, T, M)[None]
        x = rng.standard_normal((1, T)); y = rng.standard_normal((1, T))
        sx, _ = fwd(x, a)
        lty, _, _ = bwd(y, a, sx, need_grad_a=False)
        lhs = float(np.dot(y[0], sx[0])); rhs = float(np.dot(lty[0], x[0]))
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.linalg.norm(y) * np.linalg.norm(sx)), (lhs, rhs)


def check_dense_backward(fwd, bwd):
    rng = np.random.default_rng(22)
    for (T, M) in ((3, 5), (64, 5), (300, 22)):
        a = tv_coeffs(rng, T, M)
        e = rng.standard_normal(T); g = rng.standard_normal(T)
        s, _ = fwd(e[None], a[None])
        ge, ga, _ = bwd(g[None], a[None], s)
        A = dense_A(a)
        ghat = scipy.linalg.solve_triangular(A.T, g, lower=False, unit_diagonal=True)
        assert rms_rel(ge[0], ghat) < 1e-12
        s_ref = scipy.linalg.solve_triangular(A, e, lower=True, unit_diagonal=True)
        ga_ref = np.zeros((T, M))
        for t in range(T):
            for i in range(1, M + 1):
                if t - i >= 0:
                    ga_ref[t, i - 1] = -ghat[t] * s_ref[t - i]
        assert rms_rel(ga[0], ga_ref) < 1e-12


def check_ti_two_filter_gradients(fwd, bwd):
    """Eqs. 3-4 (time-invariant case): dL/de(T-t) = LP_a(g(T-t)), dL/da_i = sum_t g(t) LP_a(-s(t-i))."""
    rng = np.random.default_rng(23)
    T, M = 300, 8
    c = stable_ti_coeffs(rng, M)
    den = np.concatenate([[1.0], c])
    a = np.broadcast_to(c, (1, T, M)).copy()
    e = rng.standard_normal((1, T)); g = rng.standard_normal((1, T))
    s, _ = fwd(e, a)
    ge, ga, _ = bwd(g, a, s)
    ref_ge = scipy.signal.lfilter([1.0], den, g[0][::-1])[::-1]
    assert rms_rel(ge[0], ref_ge) < 1e-12
    for i in range(1, M + 1):
        shifted = np.zeros(T); shifted[i:] = -s[0, :T - i]
        ref = float(np.dot(g[0], scipy.signal.lfilter([1.0], den, shifted)))
        got = float(ga[0, :, i - 1].sum())
        assert abs(got - ref) <= 1e-10 * (abs(ref) + 1.0), (i, got, ref)


def check_finite_differences(fwd, bwd):
    """Central differences of L = <w, s> in float64 for e, a and zi."""
    rng = np.random.default_rng(24)
    T, M = 200, 7
    a = tv_coeffs(rng, T, M)[None]
    e = rng.standard_normal((1, T)); w = rng.standard_normal((1, T))
    zi = rng.standard_normal((1, M))

    def loss(e_, a_, zi_):
        return float(np.dot(w[0], fwd(e_, a_, zi_)[0][0]))

    s, _ = fwd(e, a, zi)
    ge, ga, gz = bwd(w, a, s, zi, need_grad_zi=True)
    h = 1e-6
    # random coordinates
    for _ in range(12):
        t = int(rng.integers(0, T)); i = int(rng.integers(0, M))
        ap = a.copy(); am = a.copy(); ap[0, t, i] += h; am[0, t, i] -= h
        fd = (loss(e, ap, zi) - loss(e, am, zi)) / (2 * h)
        assert abs(fd - ga[0, t, i]) <= 1e-6 * (abs(fd) + 1e-3), ("a", t, i, fd, ga[0, t, i])
        ep = e.copy(); em = e.copy(); ep[0, t] += h; em[0, t] -= h
        fd = (loss(ep, a, zi) - loss(em, a, zi)) / (2 * h)
        assert abs(fd - ge[0, t]) <= 1e-6 * (abs(fd) + 1e-3), ("e", t, fd, ge[0, t])
    # random directions
    for _ in range(3):
        da = rng.standard_normal(a.shape)
        fd = (loss(e, a + h * da, zi) - loss(e, a - h * da, zi)) / (2 * h)
        an = float(np.sum(ga * da))
        assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-3), (fd, an)
    for j in range(M):
        zp = zi.copy(); zm = zi.copy(); zp[0, j] += h; zm[0, j] -= h
        fd = (loss(e, a, zp) - loss(e, a, zm)) / (2 * h)
        assert abs(fd - gz[0, j]) <= 1e-6 * (abs(fd) + 1e-3), ("zi", j, fd, gz[0, j])


FORWARD_PINS = [check_golden_worked_example, check_m1_closed_forms, check_ti_lfilter,
                check_dense_forward, check_composition_expansion,
                check_linearity_and_continuation, check_state_is_past_outputs]
BACKWARD_PINS = [check_adjoint_identity, check_dense_backward, check_ti_two_filter_gradients,
                 check_finite_differences]
ALL_PINS = FORWARD_PINS + BACKWARD_PINS
