"""Host-side pieces of bench.py (no GPU): the multi-GPU refusal and the
rule that counter-derived figures are used only for the kernel sources
they were recorded for."""
from __future__ import annotations

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_recorded_profile_follows_the_source_hash(monkeypatch):
    name = "counters_rpsls_L3200.json"
    rec = bench.recorded_profile(name)
    if rec is not None:  # recorded for these very sources
        assert rec["hbm_bytes_per_launch"] > 0
        assert rec["valu_lane_ops_per_launch"] > 0
        assert rec["algorithmic_bytes_per_launch"] == 2.0 * 3200 ** 2 * 1000
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.recorded_profile(name) is None
    assert bench.recorded_profile("no_such_profile.json") is None
