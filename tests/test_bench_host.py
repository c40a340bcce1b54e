"""Host-side contract of bench.py (no GPU): the one-GPU guard, the refusal
to run without a HIP device, and the rule that the traffic figure is
reported only for the kernel sources its counters were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.skipif(bool(os.environ.get("HIP_VISIBLE_DEVICES")) or os.path.exists("/dev/kfd"),
                    reason="a HIP device may be present")
def test_no_device_exits_nonzero_without_a_line():
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert r.stdout == ""


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "pmc.md"
    prof.write_text("# counters\n\n- traffic_bytes_per_launch.k_propose = 1234.5\n"
                    "- traffic_bytes_per_launch.k_update = 777\n"
                    "- kernel_sources_sha256 = `abc`\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda sources=None: "abc")
    assert bench.measured_traffic() == 1234.5
    assert bench.measured_traffic("k_update") == 777.0
    assert bench.measured_traffic("k_fused") is None
    assert bench.measured_traffic("k_update", schedule="4,128,1") is None  # no schedule line
    prof.write_text(prof.read_text() + "- schedule = 4,128,1\n")
    assert bench.measured_traffic("k_update", schedule="4,128,1") == 777.0
    assert bench.measured_traffic("k_update", schedule="8,256,0") is None
    # kernel instances named with their options (the path's improve steps)
    prof.write_text(prof.read_text() + "- traffic_bytes_per_launch.k_path_fused<16> improve10 = 42\n")
    assert bench.measured_traffic("k_path_fused<16> improve10", str(prof)) == 42.0
    assert bench.measured_traffic("k_path_fused<16>", str(prof)) is None
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda sources=None: "def")
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_tune_cache_holds_the_headline_schedule():
    import json
    lines = [json.loads(l) for l in open(bench.TUNE_CACHE) if l.strip()]
    assert lines and all({"key", "group", "piece", "flags", "residual"} <= set(l) for l in lines)
    assert any("|n100000|k500000|" in l["key"] and "|J4096|" in l["key"] for l in lines)


def test_source_hash_covers_the_propose_sources():
    h = bench.kernel_sources_sha256()
    assert len(h) == 64 and int(h, 16) >= 0
    for name in bench.TRAFFIC_SOURCES + bench.PATH_TRAFFIC_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1206_6409_amd", "csrc", name))
    assert bench.kernel_sources_sha256(bench.PATH_TRAFFIC_SOURCES) != h
