"""Host logic of the benchmark: the one-GPU guard, and when a committed counter summary is used
(same kernel sources, same launch shape) or ignored."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_launch_tag():
    assert bench.launch_tag(None) == "defaults"
    assert bench.launch_tag({"block": 512, "grid": 2048}) == "block=512 grid=2048"
    # a persistent grid that gives every item its own workgroup maps the work like grid 0
    assert bench.launch_tag({"block": 256, "grid": 0}, 1000) == "block=256 grid=per-item"
    assert bench.launch_tag({"block": 256, "grid": 1024}, 1000) == "block=256 grid=per-item"
    assert bench.launch_tag({"block": 256, "grid": 512}, 1000) == "block=256 grid=512"
    assert bench.launch_tag({"block": 128, "grid": 2048}, 4000, 2) == "block=128 grid=per-item"
    assert bench.launch_tag({"block": 128, "grid": 1024}, 4000, 2) == "block=128 grid=1024"
    # the LDS tile per wavefront, 0 standing for the default of 10 KiB
    assert bench.launch_tag({"block": 512, "grid": 512, "tile": 16}, 1000) == "block=512 grid=512 tile=16"
    assert bench.launch_tag({"block": 256, "grid": 0, "tile": 0}, 1000) == "block=256 grid=per-item tile=10"


@pytest.fixture
def summary(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "w_hbm_counters.txt").write_text(
        "# a comment: with a colon\n"
        "k_compass.hbm_bytes_per_launch: 1234\n"
        "k_compass.source_sha256_16: aaaa\n"
        "k_compass.launch: block=256 grid=per-item\n"
        "k_fitgrad.hbm_bytes_per_launch: 99\n"
        "k_fitgrad.source_sha256_16: bbbb\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    hashes = {"k_compass": "aaaa", "k_fitgrad": "bbbb", "k_decode": "cccc"}
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: hashes[k])
    return hashes


def test_counters_used_at_the_same_sources_and_shape(summary):
    assert bench.measured_traffic("k_compass", "w", "block=256 grid=per-item") == 1234
    # a kernel that is not autotuned records no shape
    assert bench.measured_traffic("k_fitgrad", "w") == 99


def test_counters_ignored_at_another_shape(summary):
    assert bench.measured_traffic("k_compass", "w", "block=512 grid=per-item") is None
    assert bench.measured_traffic("k_compass", "w", "defaults") is None


def test_counters_ignored_after_a_source_change(summary):
    summary["k_compass"] = "changed"
    assert bench.measured_traffic("k_compass", "w", "block=256 grid=per-item") is None


def test_missing_summary_or_field(summary):
    assert bench.measured_traffic("k_compass", "other", "block=256 grid=per-item") is None
    assert bench.measured_traffic("k_decode", "w") is None
    assert bench.measured_valu("k_compass", "w", "block=256 grid=per-item") is None


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int a; // one\n/* two */ int b;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.KERNEL_SOURCES, "k_test", ["k.hip"])
    h = bench.kernel_source_hash("k_test")
    src.write_text("int a;   // changed comment\nint b; /* another */\n")
    assert bench.kernel_source_hash("k_test") == h
    src.write_text("int a; int c;\n")
    assert bench.kernel_source_hash("k_test") != h
