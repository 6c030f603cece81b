"""Host logic of bench.py: the one-GPU contract, and the accounting its
roofline and frame HBM fraction are computed from, pinned against the
per-step byte and operation breakdowns they are built from."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_frame_bytes():
    # temporal 96, variance 13, four levels at 56 and the last at 52 (no
    # variance output); the fused separable level moves the same bytes
    b = bench.BYTES_PER_PX
    assert (b["temporal"], b["variance"], b["atrous"], b["atrous_last"]) == (96, 13, 56, 52)
    assert (b["atrous_sep"], b["atrous_sep_last"]) == (56, 52)
    assert bench.frame_bytes_per_px(5, False) == 96 + 13 + 4 * 56 + 52 == 385
    assert bench.frame_bytes_per_px(5, True) == 385
    assert bench.frame_bytes_per_px(3, False) == 96 + 13 + 2 * 56 + 52


def test_valu_peak_is_the_published_fp32_rate():
    # 157.3 TFLOP/s with an FMA counted as two flops
    assert abs(bench.VALU_PEAK_TOPS - 157.3 / 2) < 0.05


def test_atrous_op_count():
    # per non-centre tap (24 of them) 18 plain operations, a log2 and an
    # exp2; per pixel 71 plain operations, 15 reciprocals and a square root
    zero = dict(exp2=0.0, log2=0.0, rcp=0.0, sqrt=0.0)
    base = bench.atrous_ops_per_px(zero)
    assert base == 24 * 18 + 71
    for k, mult in (("exp2", 24), ("log2", 24), ("rcp", 15), ("sqrt", 1)):
        assert bench.atrous_ops_per_px(dict(zero, **{k: 1.0})) - base == mult, k


def test_traffic_only_while_the_kernel_sources_are_unchanged(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    digest = bench.source_digest(bench.ATROUS_SOURCES)
    f.write_text(f"kernel_source_sha256: {digest}\nhbm_bytes_per_launch_mean: 1234.5\n")
    assert bench.measured_traffic() == 1234.5
    f.write_text(f"kernel_source_sha256: {'0' * 64}\nhbm_bytes_per_launch_mean: 1234.5\n")
    assert bench.measured_traffic() is None
    f.unlink()
    assert bench.measured_traffic() is None
