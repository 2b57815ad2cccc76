"""Host-side pieces of bench.py that need no GPU: the error statistics it
reports and its refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_rel_error_stats_nearest_rank():
    n = 200
    ref_a = np.zeros((3, n)); ref_a[0] = 2.0
    ref_j = np.zeros((3, n)); ref_j[2] = -4.0
    ref_p = -np.ones(n)
    e = np.arange(n) * 1e-6                 # particle k has relative error k * 1e-6
    rng = np.random.default_rng(0)
    perm = rng.permutation(n)               # order must not matter
    got_a = ref_a.copy(); got_a[1] += 2.0 * e[perm]        # error orthogonal to a
    got_j = ref_j * (1 + e[perm])
    got_p = ref_p * (1 - e[perm])
    s = bench.rel_error_stats((got_a, got_j, got_p), (ref_a, ref_j, ref_p))
    # nearest rank: sorted index ceil(0.99 n) - 1 = 197
    for q in ("acc", "jerk", "pot"):
        assert abs(s[q]["p99"] - 197e-6) < 1e-12, (q, s[q])
        assert abs(s[q]["max"] - 199e-6) < 1e-12, (q, s[q])


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
