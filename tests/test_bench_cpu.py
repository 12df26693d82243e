"""Host-side pieces of bench.py: the one-GPU refusal, the committed HBM
counter figures matching the kernel sources they were taken on, and the
matrix-core instruction counts behind the roofline's issued rate."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_matches_the_sources():
    """profiles/traffic.json carries a hash of the kernel sources; the bench
    reports its figures only while they match (after a kernel change they
    are stale until the counter runs are repeated)."""
    t = bench.load_traffic()
    if not t:
        pytest.skip("HBM counter figures taken on other kernel sources")
    for k in ("cfr", "cfr_adjoint", "cfr_loss"):
        assert t.get(k, 0) > 0, k
    L, M, N, P = 16384, 32, 1024, 3054729
    taps = L * M * N
    # H written once (8 B per tap) plus the path data: within 5 % of that
    assert abs(t["cfr"] / (8 * taps + 20 * P) - 1) < 0.05
    # H and H* read, dL/dH written: 24 B per tap
    assert abs(t["cfr_loss"] / (24 * taps) - 1) < 0.05
    # the adjoint reads dL/dH at least once
    assert t["cfr_adjoint"] >= 8 * taps


def test_mfma_issued_counts():
    """Two links of 17 and 40 paths, 32 elements, 1,024 subcarriers (512
    pairs): the forward product runs ceil(P/16) path chunks in each of 4
    waves (128 pairs each, 4 tiles of 32 pairs, 12 FP16 MFMAs per tile); the
    adjoint ceil(P/32) path tiles over 32 chunks of 16 pairs, 12 per chunk."""
    off = np.array([0, 17, 57])
    assert bench.mfma_issued("cfr", off, 32, 1024) == (2 + 3) * 4 * 4 * 12
    assert bench.mfma_issued("cfr_adjoint", off, 32, 1024) == (1 + 2) * 32 * 12
    # a second 32-row element block doubles both
    assert bench.mfma_issued("cfr", off, 33, 1024) == 2 * (2 + 3) * 4 * 4 * 12
    assert bench.mfma_issued("cfr_adjoint", off, 64, 1024) == 2 * (1 + 2) * 32 * 12
