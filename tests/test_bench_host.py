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
def test_algorithmic_bytes_count_each_tensor_once(L):
    # the step moves 4(3M+5) bytes per sample (e, a, s forward; g, e, a, grad_e, grad_a
    # adjoint), each credited to exactly one kernel
    n = B * T
    chunks = -(-T // L)
    last = T - (chunks - 1) * L
    names = ("fwd_scan", "fwd_emit", "bwd_scan", "bwd_emit")
    total = sum(bench.kernel_bytes(k, B, T, M, L) for k in names)
    assert total == bench.step_bytes(B, T, M) == n * 4 * (3 * M + 5)
    # fwd_scan: e, a of the chunks that carry a transition (all but each sequence's last)
    assert bench.kernel_bytes("fwd_scan", B, T, M, L) == B * (T - last) * (4 * M + 4)
    # fwd_emit: e, a of the last chunks, and s
    assert bench.kernel_bytes("fwd_emit", B, T, M, L) == B * last * (4 * M + 4) + n * 4
    assert bench.kernel_bytes("bwd_scan", B, T, M, L) == n * (4 * M + 8)       # g, e, a
    assert bench.kernel_bytes("bwd_emit", B, T, M, L) == n * (4 * M + 4)       # grad_e, grad_a
    assert bench.kernel_bytes("fwd_carry", B, T, M, L) == 0.0


def test_training_shape_figures():
    # the figures quoted at the training shape: 872.4 MB per step, bwd_scan's share 294.9 MB
    assert round(bench.step_bytes(B, T, M) / 1e6, 1) == 872.4
    assert round(bench.kernel_bytes("bwd_scan", B, T, M, 418) / 1e6, 1) == 294.9
    assert round(bench.kernel_bytes("bwd_emit", B, T, M, 418) / 1e6, 1) == 282.6


def test_traffic_table_is_plausible():
    table = bench.TRAFFIC["bytes_by_chunk"]
    assert len(bench.TRAFFIC["sources_sha256"]) == 64
    assert table, "no counter data"
    for L, row in table.items():
        assert L % M == 0
        assert set(row) <= {"fwd_scan", "fwd_emit", "bwd_scan", "bwd_emit"}
        for k, measured in row.items():
            design = bench.kernel_design_bytes(k, B, T, M, L)
            # counters include the chunk-state side arrays; anything below the bytes the
            # kernel must move or far above them would be a bad calibration
            assert 0.99 * design <= measured <= 1.25 * design, (L, k, measured, design)
            # and never below the algorithmic share
            assert measured >= bench.kernel_bytes(k, B, T, M, L)


def test_traffic_lookup_follows_the_sources():
    L = next(iter(bench.TRAFFIC["bytes_by_chunk"]))
    got = bench.measured_traffic("bwd_scan", L)
    if bench.kernel_sources_sha256() == bench.TRAFFIC["sources_sha256"]:
        assert got == bench.TRAFFIC["bytes_by_chunk"][L]["bwd_scan"]
    else:
        assert got is None
    assert bench.measured_traffic("bwd_scan", 7) is None
    # only the four row-streaming kernels, which both carry modes launch alike
    assert bench.measured_traffic("fwd_carry", L) is None
