"""Host-side checks of bench.py's contract: one GPU only, and the counter record that
is tied to the advection kernels' code (not to their comments)."""

from __future__ import annotations

import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_kernel_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1707_05163_amd", "csrc", "advect.hip")
    d = tmp_path / "paper_1707_05163_amd" / "csrc"
    d.mkdir(parents=True)
    shutil.copy(src, d / "advect.hip")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench._advect_digest()
    text = (d / "advect.hip").read_text()
    (d / "advect.hip").write_text("// a new comment line\n" + text.replace("\n", "\n  ", 3))
    assert bench._advect_digest() == base
    (d / "advect.hip").write_text(text.replace("kBlock", "kBlock2", 1))
    assert bench._advect_digest() != base


def test_counter_record_only_for_the_default_workload():
    assert bench.measured_traffic("cfg1", False) is None
    assert bench.measured_counters("cfg1", False, 288e6) is None
    assert bench.measured_traffic("cfg3", True) is None
    if bench.COUNTERS["advect_sha256"] == bench._advect_digest():
        c = bench.measured_counters("cfg1", True, 288e6)
        assert 0.0 < c["l2_hit_rate"] < 1.0 and c["hbm_bytes_per_launch"] > 0


def test_sort_cadence_defaults(monkeypatch):
    def parsed(*argv):
        monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
        return bench.parse().sort_every
    assert parsed() == bench.SORT_EVERY["cfg1"]
    assert parsed("--config", "cfg2") == bench.SORT_EVERY["cfg2"]
    assert parsed("--config", "foram") == bench.SORT_EVERY["foram"]
    # the gather kernel and RKF45 sort every segment; an explicit value always wins
    assert parsed("--stencil-cache", "0") == 1
    assert parsed("--kernel", "rkf45") == 1
    assert parsed("--config", "cfg3") == 1
    assert parsed("--sort-every", "3") == 3
