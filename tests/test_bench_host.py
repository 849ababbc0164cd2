"""Host-side pieces of bench.py, on the CPU: the one-GPU guard, the
algorithmic byte and flop counts its rooflines divide by, and the rule that
a committed traffic summary counts only for the kernel source it was taken
from."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_strip_bytes_per_frame():
    # three rows of RGB per horizontal strip, nine bytes per row per vertical strip
    assert bench.strip_bytes_per_frame(1920, 1080, 32, 32) == 32 * 3 * 5760 + 32 * 1080 * 9
    assert bench.strip_bytes_per_frame(1920, 1080, 32, 32) == 864_000
    assert bench.strip_bytes_per_frame(640, 480, 16, 16) == 161_280
    assert bench.strip_bytes_per_frame(640, 480, 16, 0) == 16 * 3 * 1920


def test_learned_flops_per_frame():
    # 12,176 multiply-adds per strip position (four width-5 convolutions and
    # the 1x1 layer), every position of 32 rows and 32 columns
    macs = 5 * (24 * 16 + 16 * 32 + 32 * 32 + 32 * 16) + 16
    assert macs == 12_176
    assert bench.cnn_flops_per_frame(1920, 1080, 32, 32) == 2.0 * macs * (32 * 1920 + 32 * 1080)


def test_learned_2d_flops_per_frame():
    # 9,896 multiply-adds per strip position: the band narrows by two lines
    # per 3x3 layer (5, 3, 1 lines of 8, 16, 32 outputs), then the 1x1 layer
    macs = 5 * 8 * 45 + 3 * 16 * 72 + 32 * 144 + 32
    assert macs == 9_896
    assert bench.cnn2d_flops_per_frame(1920, 1080, 32, 32) == 2.0 * macs * (32 * 1920 + 32 * 1080)


def test_ransac_flops_counts_frames_with_three_points():
    # the method: one squared distance (5 flops) per attempt, point and pass
    assert bench.ransac_flops([0, 2], 1024, 3) == 0.0
    assert bench.ransac_flops([100], 1024, 3) == 1024 * 100 * 4 * 5
    assert bench.ransac_flops([100, 7], 256, 0) == 256 * 107 * 5
    # the kernel's issued FP64 operations, reported beside
    assert bench.ransac_issued_flops([100], 1024, 3) == 1024 * 100 * (3 * 23 + 9)


def test_graph_calls_cover_every_context_and_batch():
    # 20 steps over 4 contexts: graphs of 5 calls, 4 launches (one per
    # context, each on a batch of its own)
    assert bench.graph_calls(20, 10, 4) == 5
    assert bench.graph_calls(1000, 10, 4) == 10
    assert bench.graph_calls(100, 10, 4) == 10
    assert bench.graph_calls(7, 10, 4) == 1
    assert bench.graph_calls(20, 10, 20) == 1
    for K in (1, 5, 20, 37, 100, 1000):
        for cycle in (1, 4, 20):
            G = bench.graph_calls(K, 10, cycle)
            assert K % G == 0
            assert K // G >= cycle or G == 1
    assert bench.rotation_used(20, 4, 5) == {"contexts": 4, "batches": 5}
    assert bench.rotation_used(4, 4, 5) == {"contexts": 4, "batches": 4}
    assert bench.rotation_used(2, 4, 5) == {"contexts": 2, "batches": 2}


def _fake_tree(tmp_path, source: bytes, recorded_sha: str):
    src = tmp_path / "paper_2210_14771_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "ca_kernels.hip").write_bytes(source)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_strips_64x1080p_hbm_traffic.md").write_text(
        "traffic_bytes_per_launch k_strips 123456\n"
        f"source_sha256_prefix {recorded_sha}\n")


def test_traffic_summary_counts_only_for_its_source(tmp_path, monkeypatch):
    source = b"// kernels\n"
    sha = hashlib.sha256(source).hexdigest()[:16]
    _fake_tree(tmp_path, source, sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_strips") == 123456
    (tmp_path / "paper_2210_14771_amd" / "csrc" / "ca_kernels.hip").write_bytes(source + b"x")
    assert bench.measured_traffic("k_strips") is None


def test_traffic_summary_missing(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_strips") is None


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))


def test_strip_kernel_name_follows_the_pairing_rule():
    # strips go in pairs when both counts are even and a workgroup takes one item
    assert bench.strip_kernel(32, 32) == "k_strips_pair"
    assert bench.strip_kernel(16, 0) == "k_strips_pair"
    assert bench.strip_kernel(32, 31) == "k_strips"
    assert bench.strip_kernel(32, 32, tiles=2) == "k_strips"


def test_contexts_in_flight_keep_graphs_of_four_calls():
    # 1000 steps: six contexts with 10-call graphs; 20 steps: five with 4-call
    # graphs rather than six with 2-call ones; every context always runs
    assert bench.contexts_in_flight(1000, 6, 10) == 6
    assert bench.contexts_in_flight(20, 6, 10) == 5
    assert bench.graph_calls(20, 10, 5) == 4
    for steps in (1, 3, 5, 7, 20, 33, 100):
        c = bench.contexts_in_flight(steps, 6, 10)
        assert 1 <= c <= min(6, steps)
        assert steps // bench.graph_calls(steps, 10, c) >= c
