"""Host-side checks of the benchmark script (no GPU): the one-GPU guard, the
algorithmic counts its roofline figures rest on, and the frame-level mixed
roofline's compulsory bytes against the workload's definition (each camera
frame read once, the panorama written once, then read and written again by
the balance)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2308_09209_amd.scenes import WORKLOADS  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_frame_roofline_compulsory_bytes_4x1080p():
    wl = WORKLOADS["4x1920x1080_ring"]
    fr = bench.frame_roofline(wl, 1080, 6144, flow_flops=0, flow_peak_tflops=157.3, ms_per_frame=1.0)
    frames = 4 * 1920 * 1080 * 3
    pano = 6144 * 1080 * 3
    assert fr["compulsory_bytes"] == frames + 3 * pano == 84_602_880
    # 84.6 MB at 8 TB/s
    assert fr["bytes_ms"] == pytest.approx(84_602_880 / 8e12 * 1e3, abs=1e-5)
    assert fr["flops_ms"] == 0 and fr["frac"] == pytest.approx(fr["bytes_ms"], abs=1e-4)


def test_frame_roofline_adds_the_flow_term():
    wl = WORKLOADS["4x1920x1080_ring"]
    a = bench.frame_roofline(wl, 1080, 6144, flow_flops=0, flow_peak_tflops=157.3, ms_per_frame=2.0)
    b = bench.frame_roofline(wl, 1080, 6144, flow_flops=157.3e9, flow_peak_tflops=157.3, ms_per_frame=2.0)
    # 157.3 GFLOP at 157.3 TFLOP/s is one millisecond
    assert b["flops_ms"] == pytest.approx(1.0)
    assert b["t_roof_ms"] == pytest.approx(a["t_roof_ms"] + 1.0, abs=1e-4)
    assert b["frac"] == pytest.approx(b["t_roof_ms"] / 2.0, abs=1e-4)
