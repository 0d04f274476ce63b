"""ctypes binding of libtvlp.so (the C ABI of include/tvlp.h).

Argument marshalling only: every step of the filter runs in the HIP kernels.
The shared library must have been built (``python -m paper_2406_05128_amd.build``
or ``__graft_entry__.build()``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtvlp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "tvlp.h")

LP_OK, LP_PENDING, LP_EINVAL, LP_ENOMEM, LP_EDEVICE, LP_ENOTFOUND, LP_EBUDGET = 0, 1, -1, -2, -3, -4, -5
LP_FLAG_NONE, LP_FLAG_CHAINED_CARRY, LP_FLAG_HIGH_RADIUS = 0, 1, 2
_CODES = {LP_EINVAL: "LP_EINVAL", LP_ENOMEM: "LP_ENOMEM", LP_EDEVICE: "LP_EDEVICE",
          LP_ENOTFOUND: "LP_ENOTFOUND", LP_EBUDGET: "LP_EBUDGET"}


class TvlpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_INT = ctypes.c_int
_SZ = ctypes.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "lp_version": (ctypes.c_char_p, []),
    "lp_last_error": (ctypes.c_char_p, []),
    "lp_supported_orders": (_INT, [_P, _INT]),
    "lp_plan_create": (_INT, [ctypes.POINTER(_P), _INT, _INT, _INT]),
    "lp_plan_destroy": (_INT, [_P]),
    "lp_plan_set_chunk": (_INT, [_P, _INT]),
    "lp_plan_get_chunk": (_INT, [_P]),
    "lp_plan_set_carry": (_INT, [_P, _INT]),
    "lp_plan_get_carry": (_INT, [_P]),
    "lp_plan_reserve": (_INT, [_P, _I64, _I64]),
    "lp_plan_autotune": (_INT, [_P, _I64, _I64, _INT, _P, _P]),
    "lp_plan_set_timing": (_INT, [_P, _INT]),
    "lp_plan_timings": (_INT, [_P, _P, _INT, _P, _P, _INT]),
    "lp_plan_reset_timings": (_INT, [_P]),
    "lp_plan_status": (_INT, [_P]),
    "lp_saved_bytes": (_SZ, [_P, _I64, _I64]),
    "lp_saved_bytes_varlen": (_SZ, [_P, _I64, _I64]),
    "lp_forward": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_forward_noalloc": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_backward": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_forward_ti": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "lp_backward_ti": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_frames_count": (_I64, [_I64, _I64]),
    "lp_coef_frames_count": (_I64, [_I64, _I64]),
    "lp_sf_last_error": (ctypes.c_char_p, []),
    "lp_sf_source": (_INT, [_I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "lp_sf_source_adjoint": (_INT, [_I64, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_fir": (_INT, [_I64, _I64, _I64, _P, _P, _P, _P]),
    "lp_fir_adjoint_work_bytes": (_SZ, [_I64, _I64, _I64]),
    "lp_fir_adjoint": (_INT, [_I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "lp_forward_frames": (_INT, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "lp_backward_frames": (_INT, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_frames_gather": (_INT, [_I64, _I64, _I64, _P, _P, ctypes.c_int, _P]),
    "lp_frames_overlap_add": (_INT, [_I64, _I64, _I64, _P, _P, ctypes.c_int, _P]),
    "lp_forward_varlen": (_INT, [_P, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "lp_backward_varlen": (_INT, [_P, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_forward_segments": (_INT, [_P, _I64, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "lp_serve_create": (_INT, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, _I64, ctypes.c_int]),
    "lp_serve_submit": (_INT, [_P, _I64, _P, _P, _P, _P]),
    "lp_serve_poll": (_INT, [_P, ctypes.c_uint64, _P]),
    "lp_serve_wait": (_INT, [_P, ctypes.c_uint64, ctypes.c_double, _P, _P]),
    "lp_serve_stats": (_INT, [_P, _P, _P, _P, _P, _P]),
    "lp_serve_destroy": (_INT, [_P]),
    "lp_saved_bytes_pair": (_SZ, [_P, _I64, _I64]),
    "lp_forward_pair": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "lp_backward_pair": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lp_graph_capture_pair_step": (_INT, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _INT,
                                          ctypes.POINTER(_P)]),
    "lp_graph_launch": (_INT, [_P, _P]),
    "lp_graph_destroy": (_INT, [_P]),
    "lp_forward_plain": (_INT, [_INT, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "lp_backward_plain": (_INT, [_INT, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
}

_lib = None


def header_symbols(path: str = HEADER) -> list[str]:
    """Function names declared in the public header."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libtvlp.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the filter has no non-HIP implementation)")
    # torch first: its HIP runtime must be the one libtvlp.so binds to.  Loading
    # the library first would bring in a second HIP runtime, and whichever
    # initialises second cannot open the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    msg = load().lp_last_error()
    return msg.decode() if msg else ""


def check(code: int) -> int:
    if code < 0:
        raise TvlpError(code, last_error())
    return code


def check_sf(code: int) -> int:
    """check() for the synthesiser calls, which keep their own error message."""
    if code < 0:
        msg = load().lp_sf_last_error()
        raise TvlpError(code, msg.decode() if msg else "")
    return code


_BUILD_ID = None


def build_id() -> str:
    """Short content hash of the libtvlp.so file this process loads."""
    global _BUILD_ID
    if _BUILD_ID is None:
        import hashlib
        h = hashlib.sha256()
        with open(LIB_PATH, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _BUILD_ID = h.hexdigest()[:16]
    return _BUILD_ID


def version() -> str:
    return load().lp_version().decode()


def supported_orders() -> list[int]:
    lib = load()
    n = lib.lp_supported_orders(None, 0)
    buf = (ctypes.c_int * n)()
    lib.lp_supported_orders(ctypes.cast(buf, _P), n)
    return list(buf)
