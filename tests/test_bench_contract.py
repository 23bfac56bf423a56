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
    assert bench.measured_counters("cfg1", False, 288e6, 2e-3) is None
    assert bench.measured_traffic("cfg3", True) is None
    if bench.COUNTERS["advect_sha256"] == bench._advect_digest():
        c = bench.measured_counters("cfg2", True, 1.44e9, 30e-3)
        assert 0.0 < c["l2_hit_rate"] < 1.0 and c["hbm_bytes_per_launch"] > 0
        assert 0.0 < c["valu_issue_frac"] < 1.0 and c["source"].startswith("profiles/")


def test_default_workload_is_the_3d_ten_million_particle_run(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.config == "cfg2" and a.dtype == "f32" and a.particles is None
    assert a.days is None and a.error_stride == 100 and a.host_stream == 0


def test_roofline_fields_recompute():
    spl, t = 1.44e9, 28e-3
    roof, alg = bench.roofline(spl, t, 192 + 56 / 144, bench.FLOPS_3D_STEP, 16.6e9)
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s"
    assert abs(roof["achieved"] - spl * bench.FLOPS_3D_STEP / t / 1e12) < 1e-3
    assert abs(roof["frac"] - roof["achieved"] / 78.6) < 1e-4
    assert abs(roof["traffic"] - 16.6e9 / t / 1e9) < 0.01
    assert abs(alg["alg_bytes_frac"] - spl * (192 + 56 / 144) / t / 8e12) < 1e-4
    assert abs(alg["reuse_factor"] - spl * (192 + 56 / 144) / 16.6e9) < 0.01
    assert abs(bench.VALU_ISSUE_PEAK * 128 - 78.6e12) / 78.6e12 < 1e-3


def test_sort_cadence_defaults(monkeypatch):
    def parsed(*argv):
        monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
        return bench.parse().sort_every
    assert parsed() == bench.SORT_EVERY["cfg2"]
    assert parsed("--config", "cfg1") == bench.SORT_EVERY["cfg1"]
    assert parsed("--config", "cfg2") == bench.SORT_EVERY["cfg2"]
    assert parsed("--config", "foram") == bench.SORT_EVERY["foram"]
    # the gather kernel and RKF45 sort every segment; an explicit value always wins
    assert parsed("--stencil-cache", "0") == 1
    assert parsed("--kernel", "rkf45") == 1
    assert parsed("--config", "cfg3") == 1
    assert parsed("--sort-every", "3") == 3
