"""MI355X-native differentiable time-varying linear prediction (arXiv 2406.05128, Sec. 3.2).

The filter s(t) = e(t) - sum_i a_i(t) s(t-i) and its adjoint run in hand-written
gfx950 HIP kernels behind the C ABI of include/tvlp.h (libtvlp.so in this
package).  Importing the package loads that library and fails if it is missing.
"""
from . import _lib

_lib.load()

from .ops import Plan, PairStepGraph, forward_plain, backward_plain  # noqa: E402
from .ops import coef_frames_count, frames_count, framewise_forward, framewise_backward  # noqa: E402
from .autograd import LPFunction, lp, get_plan, lp_frames, sf_synth  # noqa: E402
from .serve import Server  # noqa: E402
from .sf import SFSynth  # noqa: E402

__all__ = ["Plan", "PairStepGraph", "forward_plain", "backward_plain", "LPFunction", "lp", "get_plan", "Server",
           "lp_frames", "sf_synth",
           "SFSynth", "coef_frames_count", "frames_count", "framewise_forward", "framewise_backward"]
__version__ = "0.1.0"
