"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and the bench.

This package draws random numbers and builds LP coefficient tracks from
reflection coefficients.  It holds none of the filter's own arithmetic (no
recursion, no gradient): the oracle and the HIP path each implement that on
their own.
"""
from .inputs import *  # noqa: F401,F403
