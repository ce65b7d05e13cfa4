"""Host-side checks of bench.py (no GPU): which digits run, the algorithmic
bytes each pass and the whole sort must move, and the command-line contract
(one GPU only; every workload selectable)."""
import os
import subprocess
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_active_digits():
    k = torch.from_numpy(np.array([0x1200, 0x1234, 0x12FF], dtype=np.uint16))
    assert bench.active_digits(k, 16) == [True, False]
    k = torch.from_numpy(np.full(10, 0xABCD, dtype=np.uint16))
    assert bench.active_digits(k, 16) == [False, False]
    k = torch.from_numpy(np.array([1, 1 << 19, 5], dtype=np.uint32))
    assert bench.active_digits(k, 32) == [True, False, True, False]
    k = torch.from_numpy(np.array([0, 0xFF00000000000000], dtype=np.uint64))
    assert bench.active_digits(k, 64) == [False] * 7 + [True]


def test_pass_bytes():
    # 16-bit pairs: the first pass stores the high key byte (none when it
    # is the only pass), the second reads that byte and stores only payloads
    assert bench.scatter_pass_bytes(16, 4, [True, True]) == [2 + 4 + 1 + 4, 1 + 4 + 4]
    assert bench.scatter_pass_bytes(16, 4, [False, True]) == [1 + 4 + 4]
    assert bench.scatter_pass_bytes(16, 4, [True, False]) == [2 + 4 + 4]
    assert bench.scatter_pass_bytes(32, 4, [True] * 4) == [16] * 4
    assert bench.scatter_pass_bytes(64, 0, [True, False] * 4) == [16] * 4


def test_whole_sort_bytes():
    assert bench.algorithmic_bytes_per_key(16, 0, [True, True]) == 4
    # histogram read, both passes, the expansion's key write
    assert bench.algorithmic_bytes_per_key(16, 4, [True, True]) == 2 + 11 + 9 + 2
    # only the second pass: plus the high-byte copy (read 2, write 1)
    assert bench.algorithmic_bytes_per_key(16, 4, [False, True]) == 2 + 9 + 2 + 3
    assert bench.algorithmic_bytes_per_key(16, 4, [False, False]) == 2 + 8 + 2
    assert bench.algorithmic_bytes_per_key(32, 4, [True, True, False, False]) == 4 + 2 * 16
    assert bench.algorithmic_bytes_per_key(64, 8, [False] * 8) == 8 + 2 * 16


def test_more_than_one_gpu_is_refused_with_a_message():
    """The benchmark measures one GPU: --gpus N > 1 exits (status 2) with a
    message before touching any device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_new_workloads_are_selectable():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("c0", "c1", "c2a", "c2b", "c3", "c4", "c8", "wide128", "stream16", "host32"):
        assert w in r.stdout, w
