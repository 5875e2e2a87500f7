"""Host-side pieces of bench.py: the flop model and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n,flops", [(16, 43221), (32, 256427), (48, 757056), (64, 1651541)])
def test_flop_model_values(n, flops):
    assert round(bench.flop_model(n)) == flops


@pytest.mark.parametrize("n", [3, 4, 5, 17, 33, 48, 63, 64])
def test_merge_tree_partitions(n):
    merges = bench.merge_tree(n)
    # a binary tree over n leaves-of-size<=2 has (#leaves - 1) merges
    leaves = []

    def walk(d, j):
        lo, hi = (j * n) >> d, ((j + 1) * n) >> d
        if hi - lo <= 2:
            leaves.append(hi - lo)
            return
        walk(d + 1, 2 * j)
        walk(d + 1, 2 * j + 1)

    walk(0, 0)
    assert sum(leaves) == n and all(1 <= s <= 2 for s in leaves)
    assert len(merges) == len(leaves) - 1
    assert all(m == m1 + m2 and m1 >= 1 and m2 >= 1 for m, m1, m2 in merges)


def test_even_split_gemm_term_is_cubic():
    # m = 2 m1: 2 m (m1^2 + m2^2) = m^3
    assert sum(2 * m * (a * a + b * b) for m, a, b in bench.merge_tree(64)) == \
        sum(m ** 3 for m, _, _ in bench.merge_tree(64))


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
