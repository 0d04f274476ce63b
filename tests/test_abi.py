"""The C-ABI library loads and exports what include/tvlp.h declares (CPU only, no compute)."""
import ctypes

import pytest

from paper_2406_05128_amd import _lib


def test_library_exports_every_header_symbol():
    lib = _lib.load()
    declared = _lib.header_symbols()
    assert "lp_forward" in declared and "lp_backward" in declared
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows every declared call
    assert set(declared) <= set(_lib.SIGNATURES), set(declared) - set(_lib.SIGNATURES)


def test_version_and_orders():
    assert "gfx950" in _lib.version()
    orders = _lib.supported_orders()
    assert sorted(orders) == [1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 22, 24, 32]


@pytest.mark.parametrize("M", [0, 65, -3, 5, 40, 64])
def test_plan_rejects_bad_order(M):
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.lp_plan_create(ctypes.byref(h), 0, M, 0)
    assert rc == _lib.LP_EINVAL
    assert "order" in _lib.last_error()


def test_plan_rejects_unknown_flags():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.lp_plan_create(ctypes.byref(h), 0, 22, 4) == _lib.LP_EINVAL
    assert "flags" in _lib.last_error()
    assert not h.value


def test_plan_rejects_uncompiled_order():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.lp_plan_create(ctypes.byref(h), 0, 5, 0) == _lib.LP_EINVAL
    assert "compiled" in _lib.last_error()


def test_null_plan_and_bad_sizes_are_errors():
    lib = _lib.load()
    assert lib.lp_saved_bytes(None, 4, 100) == 0
    assert lib.lp_forward(None, 1, 1, None, None, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_forward_noalloc(None, 1, 1, None, None, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_backward(None, 1, 1, None, None, None, None, None, None, None, None, None, None,
                           None) == _lib.LP_EINVAL
    assert lib.lp_forward_plain(0, 1, 1, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_forward_plain(16, 0, 1, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_forward_plain(16, 1, 1, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_backward_plain(16, 1, 1, None, None, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_plan_destroy(None) == _lib.LP_OK
    assert lib.lp_plan_set_carry(None, 1) == _lib.LP_EINVAL
    assert lib.lp_plan_get_carry(None) == -1


def test_segments_pair_graph_and_server_argument_errors():
    """Argument checks that return before any device call."""
    lib = _lib.load()
    assert lib.lp_forward_segments(None, 1, None, None, 10, 0, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert "starts" in _lib.last_error()
    assert lib.lp_forward_pair(None, 1, 1, None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_graph_launch(None, None) == _lib.LP_EINVAL
    assert lib.lp_graph_destroy(None) == _lib.LP_OK
    h = ctypes.c_void_p()
    assert lib.lp_serve_create(None, 0, 16, 1 << 20, 4, 0, 0) == _lib.LP_EINVAL
    for slots in (0, -1, 5000):
        assert lib.lp_serve_create(ctypes.byref(h), 0, 16, 1 << 20, slots, 0, 0) == _lib.LP_EINVAL
        assert "max_slots" in _lib.last_error()
        assert not h.value
    t = ctypes.c_uint64()
    assert lib.lp_serve_submit(None, 10, None, None, None, ctypes.byref(t)) == _lib.LP_EINVAL
    assert lib.lp_serve_poll(None, 1, None) == _lib.LP_EINVAL
    assert lib.lp_serve_wait(None, 1, 0.0, None, None) == _lib.LP_EINVAL
    assert lib.lp_serve_stats(None, None, None, None, None, None) == _lib.LP_EINVAL
    assert lib.lp_serve_destroy(None) == _lib.LP_OK
