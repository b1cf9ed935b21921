"""Host logic of bench.py (no GPU): the one-GPU refusal and the oracle-checked count."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_oracle_checked_counts_defect_and_cost():
    # oracle: (defect, cost) per sampled instance; the GPU's info rows hold defect in column 6 and
    # cost in column 7
    ref = [(1e-6, 10.0), (2e-6, -4.0), (5e-5, 3.0), (1e-6, 7.0)]
    cpu = {"value": 1.0, "_per_instance": ref}
    info = np.zeros((6, 12))
    info[:4, 6] = [9e-6, 1e-6, 1e-6, 2e-5]               # last: the GPU misses the defect bound
    info[:4, 7] = [10.0 * (1 + 5e-4), -4.0 * (1 - 2e-3), 3.0, 7.0]
    out = bench.oracle_checked(cpu, info)
    assert "_per_instance" not in cpu                      # removed from the printed baseline
    assert out["defect_and_cost_within_1e-3"] == "1/4"     # 0 passes; 1 cost off; 2 oracle misses; 3 GPU misses
    assert out["oracle_defect_le_1e-5"] == "3/4"
    assert abs(out["cost_rel_diff_max"] - 2e-3) < 1e-12
    assert bench.oracle_checked(None, info) is None
    assert bench.oracle_checked({"value": 1.0}, info) is None
