"""The torch builder of large coefficient tracks follows the host recipe (CPU run of the same code)."""
import numpy as np
import pytest

from synth import draw_reflection_frames, make_coeffs
from synth.device import coeffs_from_frames

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("family,gamma", [("iid", 1.0), ("randomwalk", 0.995), ("ti", 0.98)])
def test_device_builder_matches_host_recipe(family, gamma):
    B, T, M = 3, 1000, 8
    a_host = make_coeffs(np.random.default_rng(5), B, T, M, 0.9, gamma, family)
    kf = draw_reflection_frames(np.random.default_rng(5), B, T, M, 0.9, family)
    a_dev = coeffs_from_frames(kf, T, gamma, "cpu", seqs_per_pass=2).numpy()
    assert a_dev.shape == a_host.shape and a_dev.dtype == np.float32
    assert np.max(np.abs(a_dev - a_host)) <= 1e-6 * max(1.0, float(np.max(np.abs(a_host))))
