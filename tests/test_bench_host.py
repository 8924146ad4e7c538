"""Host logic of the benchmark script (no GPU): the command-line contract for
several GPUs, the amortization count of Eq. (2), and the source hash that
keys the committed HBM counter records (a counter record stays valid across
edits of comments only)."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_amortization_count():
    # Eq. (2): t_pre / (t_plain - t_sel); never when the plan is not faster
    assert bench.n_iters_min(3.0, 0.5, 0.2) == pytest.approx(10.0)
    assert bench.n_iters_min(3.0, 0.2, 0.2) is None
    assert bench.n_iters_min(3.0, 0.2, 0.3) is None


def test_source_hash_ignores_comments_only():
    code = "int f(int a) {\n    return a + 1;  // one more\n}\n/* block\n comment */\n"
    base = bench.kernel_source_sha([code])
    assert bench.kernel_source_sha([code.replace("one more", "plus one")]) == base
    assert bench.kernel_source_sha([code.replace("block", "other")]) == base
    assert bench.kernel_source_sha([code.replace("    return", "\treturn")]) == base
    assert bench.kernel_source_sha([code.replace("a + 1", "a + 2")]) != base
    assert bench.kernel_source_sha([code, code]) != base

