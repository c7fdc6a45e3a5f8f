"""Host logic of the benchmark: the counter figures it reports (HBM traffic,
FP64 instructions) come from the committed profile only while the kernel
sources hash to the profiled version, and a request for more than one GPU
ends with a message instead of a number."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def write_profile(path, sha, traffic="123456789", fp64="987654321"):
    with open(path, "w") as f:
        f.write("# a profile\n\nsome text: not a field\n")
        if traffic is not None:
            f.write("traffic_bytes_per_launch: %s\n" % traffic)
        if fp64 is not None:
            f.write("fp64_wave_instructions_per_launch: %s\n" % fp64)
        f.write("kernel_source_sha256: %s\n" % sha)


def test_profile_figures_follow_the_source_hash(tmp_path, monkeypatch):
    p = tmp_path / "profile.md"
    monkeypatch.setattr(bench, "PROFILE", str(p))
    write_profile(p, bench.kernel_source_hash())
    assert bench.profiled("traffic_bytes_per_launch") == 123456789
    assert bench.profiled("fp64_wave_instructions_per_launch") == 987654321
    # another source hash: the figures were taken on other kernels
    write_profile(p, "0" * 64)
    assert bench.profiled("traffic_bytes_per_launch") is None
    # a field the profile does not hold
    write_profile(p, bench.kernel_source_hash(), fp64=None)
    assert bench.profiled("fp64_wave_instructions_per_launch") is None
    assert bench.profiled("traffic_bytes_per_launch") == 123456789


def test_missing_profile_gives_no_figures(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "absent.md"))
    assert bench.profiled("traffic_bytes_per_launch") is None


def test_source_hash_covers_the_kernel_sources(tmp_path, monkeypatch):
    a, b = tmp_path / "a.hip", tmp_path / "b.hpp"
    a.write_text("kernel one\n")
    b.write_text("header\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a), str(b)])
    h0 = bench.kernel_source_hash()
    a.write_text("kernel two\n")
    assert bench.kernel_source_hash() != h0
    a.write_text("kernel one\n")
    assert bench.kernel_source_hash() == h0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")
