"""Segment-table forward and the continuous-batching server vs the float64 oracle.

Same tolerance as the other parity tests (per sequence rms-relative error
<= 1e-4 on bandwidth-expanded inputs).  The server's scheduling must not change
a job's result: a job run among others is bit-identical to the same job run
alone through a server with the same slice length.
"""
import numpy as np
import pytest

import oracle
from synth import make_coeffs, make_excitation, poisson_requests
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
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def job(rng, T, M, kappa=0.9, gamma=0.98):
    a = make_coeffs(rng, 1, T, M, kappa, gamma, "iid")[0]
    e = make_excitation(rng, 1, T)[0]
    return e, a


# ---------------------------------------------------------------- segment tables

def _segment_layout(rng, lens, gap_max=300):
    """Non-overlapping segments placed in shuffled order with random gaps."""
    order = rng.permutation(len(lens))
    starts = np.zeros(len(lens), dtype=np.int64)
    pos = 0
    for b in order:
        pos += int(rng.integers(0, gap_max))
        starts[b] = pos
        pos += int(lens[b])
    return starts, pos + int(rng.integers(0, gap_max))


@pytest.mark.parametrize("M,L", [(22, 264), (16, 32), (4, 8)])
def test_segments_match_oracle(tv, M, L):
    rng = np.random.default_rng(11 + M)
    lens = np.array([0, 1, L - 1, L, L + 1, 3 * L + 5, 2000, 0, 777], dtype=np.int64)
    B = len(lens)
    starts, N = _segment_layout(rng, lens)
    e = np.zeros(N, np.float32)
    a = np.zeros((N, M), np.float32)
    jobs = [job(rng, max(int(n), 1), M) for n in lens]
    for b in range(B):
        n = int(lens[b])
        e[starts[b]:starts[b] + n] = jobs[b][0][:n]
        a[starts[b]:starts[b] + n] = jobs[b][1][:n]
    zi = rng.standard_normal((B, M)) * 0.1
    plan = tv.Plan(M, dev(), L)
    state = to_dev(zi.copy())
    s_sentinel = torch.full((N,), 12345.0, dtype=torch.float32, device=dev())
    s = plan.forward_segments(to_dev(e), to_dev(a), to_dev(starts), to_dev(lens), state=state, s=s_sentinel)
    plan.check_status()
    s_h = s.cpu().numpy()
    z_h = state.cpu().numpy()
    covered = np.zeros(N, bool)
    for b in range(B):
        n = int(lens[b])
        if n == 0:
            assert np.array_equal(z_h[b], zi[b]), "idle sequence's state must be untouched"
            continue
        covered[starts[b]:starts[b] + n] = True
        s_ref, zf_ref = oracle.lp_forward(e[None, starts[b]:starts[b] + n], a[None, starts[b]:starts[b] + n],
                                          zi[b:b + 1])
        assert rms_rel(s_h[starts[b]:starts[b] + n], s_ref[0]) <= TOL, (b, n)
        assert rms_rel(z_h[b], zf_ref[0]) <= TOL, (b, n)
    assert np.all(s_h[~covered] == 12345.0), "samples outside every segment must not be written"


def test_segments_continue_in_slices(tv):
    """State carried in place across slices equals one pass over the whole sequence (oracle)."""
    M, L = 22, 264
    rng = np.random.default_rng(5)
    T = 20 * L + 17
    e, a = job(rng, T, M)
    plan = tv.Plan(M, dev(), L)
    e_d, a_d = to_dev(e), to_dev(a)
    state = torch.zeros((1, M), dtype=torch.float64, device=dev())
    s = torch.empty(T, dtype=torch.float32, device=dev())
    slice_len = 3 * L
    for start in range(0, T, slice_len):
        n = min(slice_len, T - start)
        plan.forward_segments(e_d, a_d, to_dev(np.array([start])), to_dev(np.array([n])), state=state, s=s,
                              total_bound=n)
    plan.check_status()
    s_ref, zf_ref = oracle.lp_forward(e[None], a[None])
    assert rms_rel(s.cpu().numpy(), s_ref[0]) <= TOL
    assert rms_rel(state.cpu().numpy()[0], zf_ref[0]) <= TOL


def test_segments_total_bound_exceeded_is_reported(tv):
    """A table holding more samples than total_bound is flagged by the next status check."""
    M, L = 16, 32
    plan = tv.Plan(M, dev(), L)
    N = 40 * L
    e = torch.zeros(N, dtype=torch.float32, device=dev())
    a = torch.zeros((N, M), dtype=torch.float32, device=dev())
    starts = to_dev(np.array([0, 20 * L]))
    lens = to_dev(np.array([20 * L, 20 * L]))
    plan.forward_segments(e, a, starts, lens, total_bound=L)
    with pytest.raises(tv._lib.TvlpError) as ei:
        plan.check_status()
    assert ei.value.code == tv._lib.LP_EINVAL
    plan.check_status()  # the flag is cleared once reported


# ---------------------------------------------------------------- server

def _run_server(tv, M, jobs, budget, slots, slice_len, arrivals=None):
    import time
    out = {}
    with tv.Server(M, budget, max_slots=slots, slice_len=slice_len) as srv:
        tickets = []
        t0 = time.perf_counter()
        for k, (e, a) in enumerate(jobs):
            if arrivals is not None:
                delay = arrivals[k] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            tickets.append(srv.submit(e, a))
        for k, t in enumerate(tickets):
            out[k] = srv.wait(t, timeout=60.0)
        stats = srv.stats()
    return out, stats


def test_server_results_match_oracle(tv):
    M = 22
    rng = np.random.default_rng(77)
    arrivals, lengths = poisson_requests(rng, 24, rate_hz=2000.0, tmin=200, tmax=30000)
    jobs = [job(rng, int(T), M) for T in lengths]
    out, stats = _run_server(tv, M, jobs, budget=64 << 20, slots=6, slice_len=4 * 264, arrivals=arrivals)
    assert stats["jobs_done"] == len(jobs)
    assert stats["queued"] == 0 and stats["active"] == 0
    for k, (e, a) in enumerate(jobs):
        s, lat = out[k]
        s_ref, _ = oracle.lp_forward(e[None], a[None])
        assert rms_rel(s, s_ref[0]) <= TOL, (k, len(e))
        assert lat > 0


def test_server_alone_equals_in_mix(tv):
    M = 16
    rng = np.random.default_rng(3)
    lens = [5000, 131, 12000, 64, 7000, 2500, 9000, 300]
    jobs = [job(rng, T, M) for T in lens]
    mixed, _ = _run_server(tv, M, jobs, budget=16 << 20, slots=3, slice_len=512)
    for k in (0, 2, 5):
        alone, _ = _run_server(tv, M, [jobs[k]], budget=16 << 20, slots=3, slice_len=512)
        assert np.array_equal(alone[0][0], mixed[k][0]), k


def test_server_budget_admission(tv):
    """An arena that holds about two jobs still completes all of them in order; a job larger than it is refused."""
    M = 22
    rng = np.random.default_rng(9)
    T = 20000
    per_sample = (M + 2) * 4
    budget = int(2.5 * T * per_sample)
    jobs = [job(rng, T, M) for _ in range(6)]
    out, stats = _run_server(tv, M, jobs, budget=budget, slots=8, slice_len=2 * 264)
    assert stats["jobs_done"] == 6
    for k, (e, a) in enumerate(jobs):
        s_ref, _ = oracle.lp_forward(e[None], a[None])
        assert rms_rel(out[k][0], s_ref[0]) <= TOL
    with tv.Server(M, budget, max_slots=2) as srv:
        big_e, big_a = job(rng, 3 * T, M)
        with pytest.raises(tv._lib.TvlpError) as ei:
            srv.submit(big_e, big_a)
        assert ei.value.code == tv._lib.LP_EBUDGET


def test_server_ticket_lifecycle(tv):
    M = 8
    rng = np.random.default_rng(1)
    with tv.Server(M, 1 << 20, max_slots=2) as srv:
        e, a = job(rng, 1000, M)
        t = srv.submit(e, a)
        s, _ = srv.wait(t, timeout=60.0)
        s_ref, _ = oracle.lp_forward(e[None], a[None])
        assert rms_rel(s, s_ref[0]) <= TOL
        lib = tv._lib.load()
        assert lib.lp_serve_poll(srv._h, t, None) == tv._lib.LP_ENOTFOUND  # retired
        assert lib.lp_serve_poll(srv._h, 999999, None) == tv._lib.LP_ENOTFOUND
