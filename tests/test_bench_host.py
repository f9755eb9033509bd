"""Host-side logic of bench.py: the algorithmic byte count behind the roofline
figure, the counter summary it reads HBM traffic from (used only for the
kernel sources and launch shape it was measured on), and the one-GPU guard."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_the_1080p_frame():
    # per pixel: binary32 RGB in (12 B) and out (12 B), label (1 B), shell map (4 B);
    # per hole pixel: the guide (8 B)
    H, W, N = 1080, 1920, 60558
    assert bench.algorithmic_bytes(1, H, W, 3, 4, N) == H * W * 29 + 8 * N == 60618864


def test_algorithmic_bytes_in_place():
    # labels and shell map for every pixel; guide, colour read and write on the hole
    assert bench.algorithmic_bytes(2, 10, 20, 3, 2, 7, inplace=True) == 400 * 5 + 7 * (8 + 12)


def _summary(tmp_path, digest, launch, traffic):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "traffic_c2_1080p.md").write_text(
        "# HBM traffic\n\n"
        f"kernel: k\nlaunch: {launch}\nsource_sha256: {digest}\n"
        f"traffic_bytes_per_launch: {traffic}\n\nnotes\n")
    return str(tmp_path)


def test_recorded_traffic_matches_sources_and_launch(tmp_path, monkeypatch):
    root = _summary(tmp_path, "abc123", "engine=0 tile=32x32", 131312430)
    monkeypatch.setattr(bench, "ROOT", root)
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "abc123")
    monkeypatch.setattr(bench, "launch_key", lambda p, H, W, C: "engine=0 tile=32x32")
    assert bench.recorded_traffic(None, 1080, 1920, 3) == 131312430


@pytest.mark.parametrize("digest,launch", [("other", "engine=0 tile=32x32"), ("abc123", "engine=1 group=8")])
def test_recorded_traffic_is_dropped_when_stale(tmp_path, monkeypatch, digest, launch):
    root = _summary(tmp_path, "abc123", "engine=0 tile=32x32", 131312430)
    monkeypatch.setattr(bench, "ROOT", root)
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    monkeypatch.setattr(bench, "launch_key", lambda p, H, W, C: launch)
    assert bench.recorded_traffic(None, 1080, 1920, 3) is None


def test_recorded_traffic_without_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic(None, 1080, 1920, 3) is None


def test_committed_summary_parses():
    """The committed summary parses; its digest is a SHA-256 of kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_c2_1080p.md")
    with open(path) as f:
        lines = dict(line.split(":", 1) for line in f.read().splitlines()
                     if line.startswith(("source_sha256:", "launch:", "traffic_bytes_per_launch:")))
    assert len(lines["source_sha256"].strip()) == 64
    assert int(lines["traffic_bytes_per_launch"]) > 0
    assert lines["launch"].strip().startswith("engine=")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
