"""Host logic of bench.py (no GPU): the one-GPU refusal, the roofline of a
one-launch step, the gating of stored traffic by the kernel sources, and
that the hashed sources cover every local header of the step kernels."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_one_launch_roofline_takes_the_step_time():
    # per-launch events lengthen a launch beyond the time per step of the
    # uninstrumented region: a one-launch step uses the smaller of the two
    r = {"kernels_ms": {"collide": 0.0800}, "ms_per_step": 0.0774, "bytes_per_update": 288.0}
    nodes = 1 << 20
    one = bench.roofline_of(r, nodes, "k", one_launch=True)
    two = bench.roofline_of(r, nodes, "k")
    assert one["kernel_ms"] == pytest.approx(0.0774)
    assert two["kernel_ms"] == pytest.approx(0.0800)
    assert one["achieved"] == pytest.approx(288.0 * nodes / 0.0774e-3 / 1e9, rel=1e-4)
    assert one["frac"] == pytest.approx(one["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    r["ms_per_step"] = 0.09  # a step longer than its launch: the launch's own time
    assert bench.roofline_of(r, nodes, "k", one_launch=True)["kernel_ms"] == pytest.approx(0.0800)


def test_stored_traffic_only_for_the_counted_sources(monkeypatch):
    h = bench.kernel_sources_hash()
    monkeypatch.setattr(bench, "TRAFFIC", {"a": {"bytes_per_launch": 123, "sources_sha256_16": h},
                                           "b": {"bytes_per_launch": 456, "sources_sha256_16": "0" * 16}})
    assert bench.traffic_of("a") == 123
    assert bench.traffic_of("b") is None
    assert bench.traffic_of("missing") is None


def test_hashed_sources_cover_the_step_kernels_headers():
    csrc = os.path.join(ROOT, "paper_1710_07486_amd", "csrc")
    todo, seen = ["kernels.hip", "nliquid.hip"], set()
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            for inc in re.findall(r'^#include "([^"]+)"', fh.read(), re.M):
                if os.path.exists(os.path.join(csrc, inc)):
                    todo.append(inc)
    assert seen <= set(bench.KERNEL_SOURCES), seen - set(bench.KERNEL_SOURCES)
