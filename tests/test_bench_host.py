"""Host-side logic of bench.py (no GPU): the counter summary is used only
for the kernel sources it was taken on, profiler detection keeps fork pools
out of profiled runs, the multi-GPU request is refused, and the byte counts
behind the roofline follow the packed-map layout."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def recorded(key):
    path = os.path.join(ROOT, "profiles", "counters_m4096.md")
    for line in open(path):
        if line.startswith(key + ":"):
            return line.split(":", 1)[1].strip().strip("`")
    raise KeyError(key)


def test_counter_summary_needs_matching_sources(monkeypatch):
    sha = recorded("source_sha1")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha)
    t = bench.counter_traffic("traffic_bytes_per_launch_k_rollout")
    assert isinstance(t, int) and t == int(recorded("traffic_bytes_per_launch_k_rollout"))
    v = bench.counter_traffic("valu_busy_k_rollout")
    assert isinstance(v, float) and 0.0 < v < 1.0
    assert bench.counter_traffic("no_such_key") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 40)
    assert bench.counter_traffic("traffic_bytes_per_launch_k_rollout") is None


def test_profiler_detection(monkeypatch):
    for k in list(os.environ):
        if k.startswith(("ROCP_", "ROCPROF")):
            monkeypatch.delenv(k)
    monkeypatch.setenv("LD_PRELOAD", "")
    assert not bench.under_profiler()
    assert bench.map_workers() >= 1
    monkeypatch.setenv("ROCP_TOOL_LIBRARIES", "x")
    assert bench.under_profiler() and bench.map_workers() == 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "--gpus 1" in r.stderr


class _Maps:
    def __init__(self, shapes, env_to_map=None):
        self.grids = [np.zeros(s, np.uint8) for s in shapes]
        self.env_to_map = list(range(len(shapes))) if env_to_map is None else env_to_map


def test_packed_map_bytes():
    # one set word, then H + 2 rows of ceil((W + 2) / 32) words, padded to 16 B
    m = _Maps([(366, 366), (64, 30)])
    w366 = 1 + 12 * 368       # 4417 words -> 4420 -> 17,680 B
    w64 = 1 + 1 * 66          # 67 words -> 68 -> 272 B
    assert bench.env_map_bytes(m) == 17680 + 272 == (w366 + 3) // 4 * 16 + (w64 + 3) // 4 * 16


def test_window_bytes_clip_at_the_map_edges():
    # rows within ceil(max(range, r)) + 2 = 102 of the robot's row, clipped
    # to rows -1..H, 12 words a row at 366 wide, plus the word in front
    cfg = {"range": 100.0, "robot_r": 3.0}
    m = _Maps([(366, 366)], env_to_map=[0, 0])
    mid = bench.env_window_bytes(m, cfg, np.array([183.5, 183.5]))
    assert mid == 2 * 4 * ((285 - 81 + 1) * 12 + 1) == 2 * 9844
    edge = bench.env_window_bytes(m, cfg, np.array([0.5, 365.5]))
    assert edge == 4 * ((102 + 1 + 1) * 12 + 1) + 4 * ((366 - 263 + 1) * 12 + 1)
