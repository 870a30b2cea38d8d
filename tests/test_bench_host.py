"""Host-side checks of the benchmark script (no GPU): the one-GPU guard, the
algorithmic counts its roofline figures rest on, and the frame-level mixed
roofline's compulsory bytes against the workload's definition (each camera
frame read once, the panorama written once, then read and written again by
the balance)."""
import os
import subprocess
import sys

import numpy as np
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


def _brute_taps(need, r):
    """every (pixel, window offset) pair that lands inside the level"""
    h, w = need.shape
    ys, xs = np.nonzero(need)
    n = 0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            n += int(((ys + dy >= 0) & (ys + dy < h) & (xs + dx >= 0) & (xs + dx < w)).sum())
    return n


def test_flow_domain_taps_against_the_oracle_domain_by_brute_force():
    # the roofline's flop count runs over the flow domain the oracle defines
    # (the overlap at level 0, the initialisation footprints above), not over
    # the strip's bounding box
    from oracle import oracle as O
    from paper_2308_09209_amd.scenes import small_scene
    s = small_scene(n_cams=3, W=160, H=96, overlap=0.3, ring=True)
    orc = O.Oracle(s.rig())
    orc.stitch(s.frames(0))
    r = orc.params.lk_radius
    some_partial = False
    for p in range(orc.n_pairs):
        for l in range(orc.params.lk_levels):
            need = orc.tap("need", p, l)
            assert bench.domain_taps(need, r) == _brute_taps(need, r)
            full = np.ones_like(need)
            assert bench.domain_taps(full, r) == bench.window_sum(need.shape[1], r) * \
                bench.window_sum(need.shape[0], r)
            some_partial |= 0 < need.sum() < need.size
    assert some_partial


def test_lk_flops_unit_is_12_per_tap_and_step_both_directions():
    class Info:
        n_pairs, lk_levels = 2, 3
        flow_taps = [[100, 40, 10], [7, 3, 1]]
    assert bench.lk_flops_per_frame(Info, 5) == 2 * (100 + 40 + 10 + 7 + 3 + 1) * 12 * 5
    assert bench.lk_flops_per_frame(Info, 5, per_tap_step=14, per_tap=6) == 2 * 161 * (6 + 14 * 5)


def test_cpu_baseline_columns_group_as_the_papers_step_table():
    st = dict(strips=1.0, moments=0.2, solve=0.01, pyramids=0.3, flow=6.0, blend=2.0, balance=0.5)
    t = bench.table4_columns(st, 2)
    assert t["table4_ms"] == dict(geometric_warping=500.0, color_correction=355.0, local_warping=3150.0,
                                  image_blending=1000.0)
    assert t["step_ms"]["flow"] == 3000.0
