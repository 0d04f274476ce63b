"""The no-allocation forward (lp_forward_noalloc) against lp_forward, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2406_05128_amd import _lib as L
    return L


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _run(lib, plan, B, T, e, a, zi, noalloc):
    M = plan.M
    dev = e.device
    s = torch.full((B, T), float("nan"), dtype=torch.float32, device=dev)
    zf = torch.full((B, M), float("nan"), dtype=torch.float64, device=dev)
    saved = torch.zeros(plan.saved_bytes(B, T), dtype=torch.uint8, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    fn = lib.lp_forward_noalloc if noalloc else lib.lp_forward
    rc = fn(plan.handle, B, T, _vp(e), _vp(a), _vp(zi), _vp(s), _vp(zf), _vp(saved), None, st)
    return rc, s, zf, saved


@pytest.mark.parametrize("M,chunk", [(22, None), (16, 96)])
def test_noalloc_forward_equals_forward_on_two_calls(M, chunk):
    import paper_2406_05128_amd as tv
    from synth import make_coeffs, make_excitation
    L = _lib()
    lib = L.load()
    dev = torch.device("cuda", 0)
    plan = tv.Plan(M, dev, chunk)
    rng = np.random.default_rng(808 + M)
    # two calls in a row on the same plan and scratch, the second smaller (and with an initial state)
    for B, T, with_zi in ((16, 20000, False), (3, 2345, True)):
        print(f"no-alloc forward M={M} chunk={plan.chunk} B={B} T={T} zi={with_zi}", flush=True)
        e = torch.from_numpy(make_excitation(rng, B, T)).to(dev)
        a = torch.from_numpy(make_coeffs(rng, B, T, M, 0.9, 0.98)).to(dev)
        zi = torch.from_numpy(rng.standard_normal((B, M))).to(dev) if with_zi else None
        rc0, s0, zf0, sv0 = _run(lib, plan, B, T, e, a, zi, noalloc=False)
        assert rc0 == L.LP_OK, L.last_error()
        rc1, s1, zf1, sv1 = _run(lib, plan, B, T, e, a, zi, noalloc=True)
        assert rc1 == L.LP_OK, L.last_error()
        torch.cuda.synchronize()
        assert torch.equal(s1, s0)
        assert torch.equal(zf1, zf0)
        assert torch.equal(sv1, sv0)
        # and the saved states drive the ordinary backward to the same gradients
        g = torch.ones_like(e)
        ge0, ga0, _ = plan.backward(g, a, e, sv0)
        ge1, ga1, _ = plan.backward(g, a, e, sv1)
        torch.cuda.synchronize()
        assert torch.equal(ge0, ge1) and torch.equal(ga0, ga1)


def test_noalloc_forward_rejects_a_call_beyond_the_scratch():
    import paper_2406_05128_amd as tv
    L = _lib()
    lib = L.load()
    dev = torch.device("cuda", 0)
    plan = tv.Plan(22, dev, 418)
    B, T = 64, 240000  # about 25 MB of chunk offsets and group maps: more than the 16 MiB scratch
    e = torch.zeros((B, T), dtype=torch.float32, device=dev)
    a = torch.zeros((B, T, 22), dtype=torch.float32, device=dev)
    rc, _, _, _ = _run(lib, plan, B, T, e, a, None, noalloc=True)
    assert rc == L.LP_EINVAL
    assert "scratch" in L.last_error()
    # a NULL saved buffer is refused too
    s = torch.empty((2, 100), dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    assert lib.lp_forward_noalloc(plan.handle, 2, 100, _vp(e), _vp(a), None, _vp(s), None, None, None,
                                  st) == L.LP_EINVAL
