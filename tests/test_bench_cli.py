"""bench.py pieces that need no GPU: the one-GPU rule and the algorithmic op counts."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_counts():
    import bench
    from paper_1409_4923_amd import workloads as W
    ops1, tr1, _ = bench.algorithmic_work(W.C1)
    ops2, tr2, _ = bench.algorithmic_work(W.C2)
    # three drift evaluations, one cos each
    assert tr1 == pytest.approx(3.0) and tr2 > tr1
    # the Poisson workload adds the kick test, the kick add and the rare kick draws
    assert 2.0 < ops2 - ops1 < 4.0
    # normal increments cost more main-pipe work than the three-point law
    assert bench.algorithmic_work(W.C1.with_(noise=W.NORMAL))[0] > ops1
    # the jump-adapted grid costs more than the fixed grid
    assert bench.algorithmic_work(W.C2.with_(noise=W.GAUSS | W.POISSON | W.JUMP_GRID))[0] > ops2


def test_traffic_pinned_to_sources():
    import bench
    assert len(bench.KERNEL_SOURCES_SHA256) == 64
    assert bench.TRAFFIC_BYTES_PER_LAUNCH > 0
