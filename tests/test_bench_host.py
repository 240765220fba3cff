"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic cost
model of the roofline, and the validity rule of the recorded HBM traffic."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_algorithmic_bytes_of_the_operators():
    import bench
    # 256 x 256 split squares, k = 3: 131072 cells, 197120 facets
    nbytes, flops = bench.algorithmic_cost("apply_step1_operator", 3, 131072, 197120)
    # per cell: 15 x 15 volume matrix, 21 upwind weights, 7 geometry doubles,
    # three vectors of 30 doubles, 9 int32 connectivity entries
    assert nbytes == 131072 * (8 * (225 + 21 + 7 + 90) + 36) == 364380160
    assert flops > 0
    nbytes, _ = bench.algorithmic_cost("trace_spmv", 3, 131072, 197120)
    # per facet row: 5 blocks of 4 x 4, 5 column ids, x and y (4 doubles each)
    assert nbytes == 197120 * (8 * 80 + 20 + 64) == 142714880
    assert bench.algorithmic_cost("krylov_vector", 3, 1, 1) == (None, None)


def test_recorded_traffic_is_tied_to_the_kernel_source(monkeypatch):
    import bench
    with open(bench.KERNELS_SRC, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
    rec = dict(bench.MEASURED_TRAFFIC["apply_step1_operator"])
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "apply_step1_operator", {**rec, "kernels_sha256": sha})
    assert bench.measured_traffic("apply_step1_operator") == rec["bytes_per_launch"]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "apply_step1_operator", {**rec, "kernels_sha256": "0" * 16})
    assert bench.measured_traffic("apply_step1_operator") is None
    assert bench.measured_traffic("trace_spmv") is None


def test_recorded_traffic_matches_the_committed_kernels():
    """The committed record was taken on the committed kernel source, so the
    bench line carries it (a kernel change must come with fresh counters)."""
    import bench
    assert bench.measured_traffic("apply_step1_operator") is not None
