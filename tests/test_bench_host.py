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
    # per cell: the advecting field at 36 cell points (72 doubles), 21 upwind
    # weights, 7 geometry doubles, three vectors of 30 doubles, 9 int32
    # connectivity entries
    assert nbytes == 131072 * (8 * (72 + 21 + 7 + 90) + 36) == 203948032
    assert flops > 0
    nbytes, _ = bench.algorithmic_cost("trace_spmv", 3, 131072, 197120)
    # per facet row: 5 blocks of 4 x 4, 5 column ids, x and y (4 doubles each)
    assert nbytes == 197120 * (8 * 80 + 20 + 64) == 142714880
    assert bench.algorithmic_cost("krylov_vector", 3, 1, 1) == (None, None)


def test_recorded_traffic_is_tied_to_the_kernel_source(monkeypatch):
    import bench
    rec = dict(bench.MEASURED_TRAFFIC["apply_step1_operator"])
    sha = bench.kernel_sha(rec)
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "apply_step1_operator", {**rec, "sha256": sha})
    assert bench.measured_traffic("apply_step1_operator") == rec["bytes_per_launch"]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "apply_step1_operator", {**rec, "sha256": "0" * 16})
    assert bench.measured_traffic("apply_step1_operator") is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_recorded_traffic_matches_the_committed_kernels():
    """Every committed record was taken on the committed kernel source, so the
    bench line carries it (a kernel change must come with fresh counters)."""
    import bench
    for name in bench.MEASURED_TRAFFIC:
        assert bench.measured_traffic(name) is not None, name


def test_kernel_source_extraction():
    """The hash covers exactly the named functions: their text starts at the
    template line and ends with the closing brace of the body."""
    import bench
    with open(bench.os.path.join(bench.CSRC, "kernels.hip")) as fh:
        text = fh.read()
    src = bench.function_source(text, "k_spmv")
    assert src.startswith("template <int K>\n__global__") and src.rstrip().endswith("}")
    assert src.count("{") == src.count("}")
    assert "k_jacobi" not in src


def test_preconditioner_bytes():
    import bench
    # 256 x 256, k = 3: per cell the 60 x 30 first-pass rows and the 30 x 30
    # H in FP16, two FP64 vectors, 60 FP64 first-pass results written and
    # read; per interior facet (196096) a 20 x 20 FP16 correction and two scales
    nbytes, _ = bench.algorithmic_cost("step1_precond_apply", 3, 131072, 197120, 196096)
    assert nbytes == 131072 * (60 * 30 * 2 + 30 * 30 * 2 + 2 * 8 * 30 + 2 * 8 * 60 + 12) + 196096 * (20 * 20 * 2 + 8)
    # the operator on the method's own data: 4 vectors of 30 doubles (input,
    # output, inner-product vector, Q*), 7 geometry doubles, 9 int32 entries
    assert bench.method_bytes("apply_step1_operator", 3, 131072) == 131072 * (8 * (120 + 7) + 36)
