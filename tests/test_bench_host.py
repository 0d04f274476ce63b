"""Host-side checks of bench.py: the one-GPU contract, the algorithmic byte and
FLOP model of each kernel, and the stored hardware-counter traffic table."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

B, T, M = 64, 48000, 22


def test_more_than_one_gpu_is_refused():
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 2
    assert "one GPU" in proc.stderr
    assert proc.stdout == ""


@pytest.mark.parametrize("L", [418, 506, 66, 2048])
def test_algorithmic_bytes_per_sample(L):
    # bytes per sample: coefficient row 4M, one float32 per scalar stream
    n = B * T
    chunks = -(-T // L)
    last = T - (chunks - 1) * L
    assert bench.kernel_bytes("fwd_emit", B, T, M, L) == n * (4 * M + 8)        # e, a -> s
    assert bench.kernel_bytes("bwd_scan", B, T, M, L) == n * (8 * M + 12)       # (g, a) + (e, a -> s)
    assert bench.kernel_bytes("bwd_emit", B, T, M, L) == n * (8 * M + 12)       # g, s, a -> grad_e, grad_a
    # the basis pass only runs over chunks whose transition is used: all but each sequence's last
    assert bench.kernel_bytes("fwd_scan", B, T, M, L) == B * (T - last) * (4 * M + 4)
    assert bench.kernel_bytes("fwd_carry", B, T, M, L) == 0.0


def test_training_shape_figures():
    # the figures quoted for chunk length 418 at the training shape
    assert round(bench.kernel_bytes("fwd_scan", B, T, M, 418) / 1e6, 1) == 280.6
    assert round(bench.kernel_bytes("bwd_emit", B, T, M, 418) / 1e6, 1) == 577.5
    # M + 1 recursions of M FMAs per sample in the basis pass
    assert bench.kernel_flops("fwd_scan", B, T, M, 418) == B * (T - 348) * (M + 1) * M * 2


def test_traffic_table_is_plausible():
    table = bench.TRAFFIC["bytes_by_chunk"]
    assert len(bench.TRAFFIC["sources_sha256"]) == 64
    assert table, "no counter data"
    for L, row in table.items():
        assert L % M == 0
        assert set(row) == {"fwd_scan", "fwd_emit", "bwd_scan", "bwd_emit"}
        for k, measured in row.items():
            alg = bench.kernel_bytes(k, B, T, M, L)
            # counters include the chunk-state side arrays; anything below the
            # algorithmic bytes or far above them would be a bad calibration
            assert 0.99 * alg <= measured <= 1.25 * alg, (L, k, measured, alg)


def test_traffic_lookup_follows_the_sources():
    L = next(iter(bench.TRAFFIC["bytes_by_chunk"]))
    got = bench.measured_traffic("bwd_scan", L)
    if bench.kernel_sources_sha256() == bench.TRAFFIC["sources_sha256"]:
        assert got == bench.TRAFFIC["bytes_by_chunk"][L]["bwd_scan"]
    else:
        assert got is None
    assert bench.measured_traffic("bwd_scan", 7) is None
