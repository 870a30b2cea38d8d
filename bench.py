#!/usr/bin/env python3
"""Benchmark of the per-frame stitching path on one MI355X.

One step = one frame through the whole path (pre-warp strips + histograms,
histogram specification + moments + 3D-M solve, luma pyramids, pyramidal
flow, local warp + blend, balancing) on the 4 x 1920x1080 ring (20 % overlap,
6144 x 1080 panorama, exposure drift).  Frames are generated with the seeded
scene generator, uploaded once and resident in HBM before the timed region.

Prints one JSON line: panorama Mpix/s (value), p50/p99 frame latency, per-step
device times, the roofline of the dominant kernel (the flow kernel) and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
BF16_MFMA_PEAK_TFLOPS = 2500.0    # MI355X published dense BF16 matrix peak
HBM_PEAK_TBS = 8.0                # MI355X published HBM3E bandwidth
HBM_PEAK_GBS = 8000.0
DEFAULT_WEIGHTS = os.path.join(ROOT, "paper_2308_09209_amd", "weights", "flow_surrogate.vsnn")
FLOW_MODES = {"plain": 0, "surrogate": 1, "fallback": 2}


FLOPS_PER_TAP_STEP = 12   # algorithmic unit: per window tap and Gauss-Newton step, 4 bilinear MACs,
                          # the residual and 2 right-hand-side MACs (FMA = 2 flops)


def window_sum(n, r):
    """sum over positions of the clipped window length along one axis"""
    return sum(min(x + r, n - 1) - max(x - r, 0) + 1 for x in range(n))


def domain_taps(need, r):
    """Window taps of the flow estimate over a flow domain (uint8 map, 1 where
    the flow is estimated): the sum over the marked pixels of the (2r+1)^2
    window clipped to the level."""
    h, w = need.shape
    wx = np.array([min(x + r, w - 1) - max(x - r, 0) + 1 for x in range(w)], np.int64)
    wy = np.array([min(y + r, h - 1) - max(y - r, 0) + 1 for y in range(h)], np.int64)
    return int((need.astype(bool) * wy[:, None] * wx[None, :]).sum())


def lk_flops_per_frame(info, iters, per_tap_step=FLOPS_PER_TAP_STEP, per_tap=0):
    """Algorithmic FP32 flops of the plain flow per frame: both directions of
    every pair, every level, over the planned flow domain (info.flow_taps =
    the clipped window taps of its pixels), per_tap_step flops per tap and
    Gauss-Newton step (+ per_tap once per tap for the normal matrix)."""
    total = 0
    for p in range(info.n_pairs):
        for l in range(info.lk_levels):
            total += 2 * int(info.flow_taps[p][l]) * (per_tap + per_tap_step * iters)
    return total


def load_pmc(kernel, workload):
    """HBM traffic of the kernel measured with rocprofv3 counters, if the record
    was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2308_09209_amd", "csrc", "vs_flow.hip"), "rb").read()
    if rec.get("kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("bytes_per_launch")


def frame_roofline(wl, pano_h, pano_w, flow_flops, flow_peak_tflops, ms_per_frame):
    """Frame-level mixed roofline: the time a frame would take if every step ran
    at its own bound, over the measured time.  Bytes: the compulsory ones (each
    camera frame read once, the panorama written once, then read and written
    again by the balance, which needs the frame's own histogram first) at the
    HBM peak; flops: the flow step's algorithmic count at its unit's peak.  The
    other steps' arithmetic and the declared intermediates (strips, pyramids,
    flows) are left out, so this is a lower bound on the frame time."""
    frames_b = wl["n_cams"] * wl["W"] * wl["H"] * 3
    pano_b = pano_h * pano_w * 3
    comp = frames_b + 3 * pano_b
    t_bytes = comp / (HBM_PEAK_TBS * 1e12) * 1e3
    t_flops = flow_flops / (flow_peak_tflops * 1e12) * 1e3
    t_roof = t_bytes + t_flops
    return dict(t_roof_ms=round(t_roof, 5), t_ms=round(ms_per_frame, 5), frac=round(t_roof / ms_per_frame, 4),
                compulsory_bytes=comp, bytes_ms=round(t_bytes, 5), flow_flops=int(flow_flops),
                flow_peak_tflops=flow_peak_tflops, flops_ms=round(t_flops, 5))


def surrogate_flops_per_frame(info, layers):
    """matrix-core flops of the surrogate network per frame: 2 * 9 * cin * cout
    per level-2 pixel and layer, both directions of every pair; the first
    layer counts its 2 non-zero input channels (the luma pair)"""
    per_px = sum(2 * 9 * (2 if i == 0 else ci) * co for i, (ci, co) in enumerate(layers))
    total = 0
    for p in range(info.n_pairs):
        w, h = info.strip_w[p], info.strip_h[p]
        for _ in range(2):
            w, h = (w + 1) // 2, (h + 1) // 2
        total += 2 * w * h * per_px
    return total


def blob_layers(blob):
    import struct
    nl = struct.unpack_from("<I", blob, 8)[0]
    return [struct.unpack_from("<II", blob, 16 + 8 * i) for i in range(nl)]


def time_frames(st, frames, pano, start, K):
    """Three passes over the same K frames: throughput (no event recorded on
    the stream: in kernel traces every recorded timing event leaves a gap of
    about 5 µs before the next kernel starts), latency (one event pair around
    each frame) and the library's per-step times (its own events between the
    steps of every frame)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        st.stitch(frames[(start + i) % len(frames)], pano=pano)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for i in range(K):
        starts[i].record()
        st.stitch(frames[(start + i) % len(frames)], pano=pano)
        ends[i].record()
    torch.cuda.synchronize()
    lat = np.array([starts[i].elapsed_time(ends[i]) for i in range(K)])
    st.set_timing(True)
    for i in range(K):
        st.stitch(frames[(start + i) % len(frames)], pano=pano)
    torch.cuda.synchronize()
    step_ms, nfr = st.timing()
    st.set_timing(False)
    return wall, lat, step_ms, nfr


def flow_epe(st_a, st_b):
    """mean end-point error between two contexts' level-0 flows over the
    overlap pixels, both directions of every pair (px), and its 99th percentile"""
    errs = []
    for p in range(st_a.n_pairs):
        need = st_a.tap("need", p, 0).astype(bool)
        for d in (0, 1):
            a, b = st_a.tap("flow", p, d), st_b.tap("flow", p, d)
            errs.append(np.sqrt(((a.astype(np.float64) - b) ** 2).sum(-1))[need])
    e = np.concatenate(errs)
    return float(e.mean()), float(np.percentile(e, 99))


def cpu_baseline(scene, frames_list, n_frames):
    from oracle import oracle as O
    rig = scene.rig()
    orc = O.Oracle(rig)
    H, W = orc.canvas
    t0 = time.perf_counter()
    for t in range(n_frames):
        orc.stitch(frames_list[t])
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    threads = min(threads, len(os.sched_getaffinity(0)))
    out = dict(value=round(n_frames * H * W / dt / 1e6, 4), unit="Mpix/s", cores=threads,
               kind="oracle", sample=f"{n_frames} consecutive frames of the same workload, every step "
                                     f"({dt:.1f} s on {threads} OpenMP threads)",
               cpu_model=cpu_model(), nproc=os.cpu_count(),
               **table4_columns(orc.step_times(), n_frames))
    # the next frame on one thread (the oracle's OpenMP regions follow this thread's setting)
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        gomp = None
    if gomp is not None and len(frames_list) > n_frames and H * W <= 8_000_000:   # ~10-20 s of one core
        gomp.omp_set_num_threads(1)
        before = orc.step_times()
        t0 = time.perf_counter()
        orc.stitch(frames_list[n_frames])
        dt1 = time.perf_counter() - t0
        after = orc.step_times()
        gomp.omp_set_num_threads(threads)
        out["single_thread"] = dict(value=round(H * W / dt1 / 1e6, 4), unit="Mpix/s",
                                    sample=f"1 frame ({dt1:.1f} s)",
                                    **table4_columns({k: after[k] - before[k] for k in after}, 1))
    return out


def table4_columns(step_s, n_frames):
    """Per-frame oracle step times (ms), each step and grouped as the paper's
    per-step timing table: geometric warping (strip pre-warp), colour
    correction (histogram specification, moments, solve, balancing), local
    warping (flow input pyramids and flow), image blending."""
    ms = {k: round(v / n_frames * 1e3, 2) for k, v in step_s.items()}
    return dict(step_ms=ms, table4_ms=dict(
        geometric_warping=ms["strips"],
        color_correction=round(ms["moments"] + ms["solve"] + ms["balance"], 2),
        local_warping=round(ms["pyramids"] + ms["flow"], 2),
        image_blending=ms["blend"]))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=None, help="default 4x1920x1080_ring")
    ap.add_argument("--seq", type=int, default=None,
                    help="distinct frames generated and cycled (default 60; 4 for the 8 x 3840x2160 ring, whose "
                         "frames take seconds each to synthesise)")
    ap.add_argument("--cpu-frames", type=int, default=None, help="oracle frames timed (default 3; 1 at 8 x 4K)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="the 6-stream batched workload (2x1280x720, 2x1920x1080, 2x2560x1440, "
                         "3-4 cameras each) through one captured graph, instead of the ring; with an "
                         "explicit --workload, that one workload through the captured graph")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the flow kernel and the fused pyramid's tile height first (batch)")
    ap.add_argument("--tune-records", default=None,
                    help="tuning-record file: loaded before the contexts are created (when it exists) "
                         "and, after --autotune, written back")
    ap.add_argument("--flow", choices=sorted(FLOW_MODES), default=None,
                    help="flow mode of the surrogate leg (default fallback; plain: no surrogate leg); "
                         "with --batch the flow mode of every stream (default plain)")
    ap.add_argument("--fb-tau", type=float, default=0.5,
                    help="forward-backward threshold (px) of the fallback mode")
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS, help="surrogate weight file")
    ap.add_argument("--epe-frames", type=int, default=3, help="frames compared for the surrogate's EPE")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (a "
                         "counter reference for rocprofv3 byte counters)")
    ap.add_argument("--no-variational", action="store_true", help="skip the variational-flow leg")
    ap.add_argument("--var-steps", type=int, default=100, help="frames timed in the variational-flow leg")
    ap.add_argument("--streaming-bytes", action="store_true",
                    help="only print the algorithmic bytes per dispatch of the strip, blend and balance kernels "
                         "for the 4x1080p ring, the 8x4K ring and the 6-stream batch, from their plans")
    ap.add_argument("--conv-rate", action="store_true",
                    help="only time the matrix-core 3x3 convolution on level-0 strip sizes "
                         "(8 images of 1080 x 256) for the layer shapes the library builds")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the stitching path runs on one GPU (how it would shard across GPUs is a "
              "design, not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2308_09209_amd import vstitch as V
    from paper_2308_09209_amd.scenes import WORKLOADS, scene_for

    if args.conv_rate:
        return conv_rate(V)
    if args.streaming_bytes:
        return streaming_bytes(V)
    big = args.workload == "8x3840x2160_ring"
    if args.seq is None:
        args.seq = 4 if big else 60
    if args.cpu_frames is None:
        args.cpu_frames = 1 if big else 3
    if args.batch:
        args.flow = args.flow or "plain"
        return bench_batch(args)
    args.workload = args.workload or "4x1920x1080_ring"
    args.flow = args.flow or "fallback"

    wl = WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    scene = scene_for(args.workload)
    rig = scene.rig()
    seq = max(1, args.seq)
    host_frames = []
    for t in range(seq):
        host_frames.append(scene.frames(t))
        print(f"# frame {t} generated ({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    print(f"# generated {seq} frames in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    frames = [[torch.from_numpy(f).to(dev) for f in fr] for fr in host_frames]

    if args.copy_calibration_mb > 0:
        copy_calibration(args.copy_calibration_mb, dev)

    st = V.Stitcher(rig)
    info = st.info
    H, W = st.canvas
    pano = st.new_pano(dev)
    torch.cuda.synchronize()
    for i in range(args.warmup):
        st.stitch(frames[i % seq], pano=pano)
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} frames)", file=sys.stderr, flush=True)

    K = args.steps
    wall, lat, step_ms, nfr = time_frames(st, frames, pano, args.warmup, K)
    print(f"# timed {K} frames in {wall:.3f} s", file=sys.stderr, flush=True)

    mpix = K * H * W / wall / 1e6
    levels = info.lk_levels
    p = st.params
    flops = lk_flops_per_frame(info, p.lk_iters)
    # as the kernel issues them: 5 FMA per tap once per level (normal matrix and
    # template term); per tap and step 4 FMA plus the interpolation along x
    # (1 sub + 1 FMA) of 10 moving-image rows per 9 window rows
    flops_impl = lk_flops_per_frame(info, p.lk_iters, per_tap_step=8 + 3 * 10 / 9, per_tap=10)
    taps = sum(int(info.flow_taps[q][l]) for q in range(info.n_pairs) for l in range(levels))
    lk_launch_ms = step_ms[2] / nfr / levels
    achieved = flops / levels / (lk_launch_ms * 1e-3) / 1e12
    traffic = load_pmc("k_lk", args.workload)
    roofline = dict(bound="alu", kernel="vs::k_lk_w9 + vs::k_lk_tail (pyramidal flow, one launch "
                                        "pair per level)",
                    achieved=round(achieved, 3), peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                    traffic=traffic, avg_launch_ms=round(lk_launch_ms, 5),
                    flops_per_launch=int(flops / levels),
                    unit_flops=f"{FLOPS_PER_TAP_STEP} flop per window tap and Gauss-Newton step over the "
                               f"flow domain ({taps} taps per direction per frame, {p.lk_iters} steps, "
                               "2 directions)",
                    achieved_impl_count=round(flops_impl / levels / (lk_launch_ms * 1e-3) / 1e12, 3),
                    impl_count="10 flop per tap (normal matrix, template term) + 11.33 per tap and step "
                               "(4 FMA, interpolation along x shared by two window rows), as the kernel "
                               "issues them")
    names = V.Stitcher.TIMING_STEPS
    metric = ("panorama Mpix/s + p99 frame ms, 4x1080p; surrogate vs plain flow @EPE<=0.5px"
              if args.workload == "4x1920x1080_ring" else
              f"panorama Mpix/s + p99 frame ms, {args.workload}; surrogate vs plain flow @EPE<=0.5px")
    out = dict(metric=metric, value=round(mpix, 2), unit="Mpix/s", n_gpus=1,
               steps=K, warmup=args.warmup, ms_per_step=round(wall / K * 1e3, 4),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=args.workload, cams=wl["n_cams"], frame=f"{wl['W']}x{wl['H']}",
                           overlap=wl["overlap"], ring=wl["ring"], panorama=f"{W}x{H}",
                           seq_frames=seq, flow="plain pyramidal LK (L=4, K=5, r=4, lambda=256)",
                           parallelism="single GPU"),
               p50_ms=round(float(np.percentile(lat, 50)), 4),
               p99_ms=round(float(np.percentile(lat, 99)), 4),
               step_ms={n: round(v / nfr, 5) for n, v in zip(names, step_ms)},
               roofline=roofline,
               frame_roofline=frame_roofline(wl, H, W, flops, FP32_VECTOR_PEAK_TFLOPS, wall / K * 1e3))
    if args.flow != "plain" and os.path.exists(args.weights):
        out["surrogate"] = surrogate_leg(args, V, rig, frames, st, K, H, W, mpix, float(np.percentile(lat, 99)))
    if not args.no_variational:
        out["variational"] = variational_leg(args, V, rig, frames, st, H, W, mpix)
    if not args.no_cpu_baseline:
        print(f"# timing the CPU oracle on {args.cpu_frames} frames", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(scene, host_frames, min(args.cpu_frames, seq))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def surrogate_leg(args, V, rig, frames, st_plain, K, H, W, mpix_plain, p99_plain):
    """The same frames with the learned flow surrogate: throughput, latency, its
    flows' end-point error against the plain path's, and the matrix-core rate."""
    import torch

    from paper_2308_09209_amd.scenes import WORKLOADS
    blob = open(args.weights, "rb").read()
    mode, tau = FLOW_MODES[args.flow], args.fb_tau
    ss = V.Stitcher(rig)
    ss.load_weights(blob)
    ss.set_flow_mode(mode, tau)
    pano = ss.new_pano()
    # EPE against the plain path: both contexts fed the same frames from T = 0
    ref = V.Stitcher(rig)
    epes, p99s, kept, pairs = [], [], 0, 0
    for t in range(min(args.epe_frames, len(frames))):
        ref.stitch(frames[t], pano=pano)
        _, _, info = ss.stitch(frames[t], pano=pano, want_info=True)
        e, e99 = flow_epe(ss, ref)
        epes.append(e)
        p99s.append(e99)
        kept += sum(info.surr_ok[p] for p in range(ss.n_pairs))
        pairs += ss.n_pairs
    del ref
    for i in range(args.warmup):
        ss.stitch(frames[i % len(frames)], pano=pano)
    torch.cuda.synchronize()
    wall, lat, step_ms, nfr = time_frames(ss, frames, pano, args.warmup, K)
    print(f"# surrogate ({args.flow}): timed {K} frames in {wall:.3f} s", file=sys.stderr, flush=True)
    mpix = K * H * W / wall / 1e6
    fl = surrogate_flops_per_frame(ss.info, blob_layers(blob))
    flow_ms = step_ms[2] / nfr
    names = V.Stitcher.TIMING_STEPS
    return dict(mode=args.flow, fb_tau_px=tau if mode == 2 else None, weights=os.path.basename(args.weights),
                value=round(mpix, 2), unit="Mpix/s", ms_per_step=round(wall / K * 1e3, 4),
                p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
                speedup_vs_plain=round(mpix / mpix_plain, 3),
                p99_vs_plain=round(float(np.percentile(lat, 99)) / p99_plain, 3),
                epe_vs_plain_px=round(float(np.mean(epes)), 4), epe_p99_px=round(float(np.mean(p99s)), 4),
                epe_frames=min(args.epe_frames, len(frames)), pairs_kept=f"{kept}/{pairs}",
                step_ms={n: round(v / nfr, 5) for n, v in zip(names, step_ms)},
                frame_roofline=frame_roofline(WORKLOADS[args.workload], H, W, fl, BF16_MFMA_PEAK_TFLOPS,
                                              wall / K * 1e3),
                mfma=dict(flops_per_frame=fl, flow_step_ms=round(flow_ms, 5),
                          achieved=round(fl / (flow_ms * 1e-3) / 1e12, 3), peak=BF16_MFMA_PEAK_TFLOPS,
                          unit="TFLOP/s", note="network flops (first layer on its 2 non-zero input "
                          "channels) over the whole flow step (5 convolutions, upsampling, "
                          "forward-backward check, fallback)"))


def streaming_bytes(V):
    """Algorithmic HBM bytes per dispatch of the streaming kernels, from the
    plans: k_strips 15 B per strip pixel (both cameras' source pixel read once,
    both strips and the overlap mask written), k_blend the camera frames read
    once, both flows of each overlap pixel (2 x 8 B) and the panorama written
    once, k_balance_apply the panorama read and written once."""
    from paper_2308_09209_amd.scenes import batch_scenes, scene_for
    out = {}
    for name, scs in (("4x1920x1080_ring", [scene_for("4x1920x1080_ring")]),
                      ("8x3840x2160_ring", [scene_for("8x3840x2160_ring")]), ("6stream_batch", batch_scenes())):
        tot = dict(canvas=0, strip=0, overlap=0, frames=0)
        for sc in scs:
            st = V.Stitcher(sc.rig())
            I = st.info
            tot["canvas"] += I.canvas_w * I.canvas_h
            tot["strip"] += sum(I.strip_w[p] * I.strip_h[p] for p in range(I.n_pairs))
            tot["overlap"] += sum(int(I.flow_px[p][0]) for p in range(I.n_pairs))
            tot["frames"] += sc.n_cams * sc.W * sc.H * 3
            st.close()
        out[name] = dict(pixels=tot, k_strips=15 * tot["strip"],
                         k_blend=tot["frames"] + 16 * tot["overlap"] + 3 * tot["canvas"],
                         k_balance_apply=6 * tot["canvas"])
    print(json.dumps(out), flush=True)


def copy_calibration(mib, dev):
    """one plain device-to-device copy of `mib` MiB: the reference the
    rocprofv3 byte counters are scaled by"""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    print(f"# copied {mib} MiB device to device (counter reference)", file=sys.stderr, flush=True)


def conv_rate(V, H=1080, W=256, N=8, K=20):
    """Matrix-core 3x3 convolution rate (BF16 in and out, FP32 accumulation,
    leaky ReLU) on N images of H x W -- the level-0 strips of a 4 x 1080p ring,
    both directions of its 4 pairs -- for each layer shape the library builds."""
    import ctypes as C

    import torch
    imgs = V.nn_images([(H, W)] * N)
    P = H * W * N
    out = {}
    for cin, cout in ((16, 32), (32, 32), (32, 16)):
        x = torch.randint(-16000, 16000, (P * cin,), dtype=torch.int16, device="cuda")
        w = torch.randint(-2000, 2000, (cout * 9 * cin,), dtype=torch.int16, device="cuda")
        b = torch.zeros(cout, dtype=torch.float32, device="cuda")
        y = torch.empty(P * cout, dtype=torch.int16, device="cuda")

        def run():
            V.check(V.lib().vs_nn_conv3x3(C.c_void_p(x.data_ptr()), cin, C.c_void_p(w.data_ptr()),
                                          C.c_void_p(b.data_ptr()), C.c_void_p(y.data_ptr()), cout,
                                          C.byref(imgs), V.CONV_LRELU, 0.1, None), "vs_nn_conv3x3")
        for _ in range(3):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        fl = 2.0 * 9 * cin * cout * P
        out[f"{cin}->{cout}"] = dict(ms=round(ms, 4), gflop=round(fl / 1e9, 3),
                                     tflops=round(fl / ms / 1e9, 2),
                                     frac=round(fl / ms / 1e9 / BF16_MFMA_PEAK_TFLOPS, 4))
    print(json.dumps(dict(what="3x3 convolution rate", images=f"{N} x {H}x{W}", peak=BF16_MFMA_PEAK_TFLOPS,
                          unit="TFLOP/s", layers=out)), flush=True)


def var_bytes_per_frame(info, outer, inner):
    """Algorithmic HBM bytes of the variational flow step per frame: per level
    and pair, with n the field's pixels: derivatives 2 cameras x (4 read + 20
    written), initialisation 2 directions x (8 written + 2 read), each warp 2 x
    (U 8, the moving image and its 5 derivative planes 24, T 4 and its 2
    gradient planes 8, coefficients 32 and increments 8 written; + 16 to fold
    the previous increments after the first), each Jacobi step 2 x (coefficients
    32, U 8, increments 8 and the domain mask 1 read, increments 8 written),
    the last fold 2 x 24."""
    total = 0
    for p in range(info.n_pairs):
        w, h = int(info.strip_w[p]), int(info.strip_h[p])
        for l in range(info.lk_levels):
            n = w * h
            w, h = (w + 1) // 2, (h + 1) // 2
            warps = sum(84 + (16 if o > 0 else 0) for o in range(outer))
            total += n * (2 * 24 + 2 * 10 + 2 * warps + 2 * outer * inner * 57 + 2 * 24)
    return total


def variational_leg(args, V, rig, frames, st_plain, H, W, mpix_plain):
    """The same frames with the variational flow alternative (flow = 2):
    throughput, latency, its flows' end-point error against the plain
    path's, and the flow step's rate against HBM on its algorithmic bytes."""
    sv = V.Stitcher(rig, flow=2)
    pano = sv.new_pano()
    ref = V.Stitcher(rig)
    epes, p99s = [], []
    for t in range(min(args.epe_frames, len(frames))):
        ref.stitch(frames[t], pano=pano)
        sv.stitch(frames[t], pano=pano)
        e, e99 = flow_epe(sv, ref)
        epes.append(e)
        p99s.append(e99)
    ref.close()
    for i in range(min(args.warmup, 5)):
        sv.stitch(frames[i % len(frames)], pano=pano)
    K = args.var_steps
    wall, lat, step_ms, nfr = time_frames(sv, frames, pano, args.warmup, K)
    print(f"# variational: timed {K} frames in {wall:.3f} s", file=sys.stderr, flush=True)
    p = sv.params
    flow_ms = step_ms[2] / nfr
    vb = var_bytes_per_frame(sv.info, p.var_outer, p.var_inner)
    names = V.Stitcher.TIMING_STEPS
    out = dict(flow=f"variational (L={sv.info.lk_levels}, {p.var_outer} warps x {p.var_inner} Jacobi steps, "
                    f"alpha={p.var_alpha:g}, gamma={p.var_gamma:g})",
               value=round(K * H * W / wall / 1e6, 2), unit="Mpix/s", ms_per_step=round(wall / K * 1e3, 4),
               p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
               vs_plain=round(K * H * W / wall / 1e6 / mpix_plain, 3),
               epe_vs_plain_px=round(float(np.mean(epes)), 4), epe_p99_px=round(float(np.mean(p99s)), 4),
               epe_frames=min(args.epe_frames, len(frames)),
               step_ms={n: round(v / nfr, 5) for n, v in zip(names, step_ms)},
               roofline=dict(bound="hbm", kernel="vs::k_var_* (the whole variational flow step)",
                             achieved=round(vb / (flow_ms * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(vb / (flow_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), traffic=None,
                             bytes_per_frame=vb,
                             unit_bytes="per level and field pixel: derivatives, initialisation, warps and "
                                        "Jacobi steps (57 B each: coefficients, flow, increments, mask read; "
                                        "increments written), fold"))
    sv.close()
    return out


IN_FLIGHT = 3


def bench_batch(args):
    import torch

    from paper_2308_09209_amd import vstitch as V
    from paper_2308_09209_amd.scenes import BATCH_STREAMS, WORKLOADS, batch_scenes, scene_for

    t_gen = time.perf_counter()
    scenes = [scene_for(args.workload)] if args.workload else batch_scenes()
    seq = max(1, args.seq)
    dev = torch.device("cuda:0")
    frames = []
    for t in range(seq):
        frames.append([[torch.from_numpy(f).to(dev) for f in sc.frames(t)] for sc in scenes])
        print(f"# frame {t} generated ({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    print(f"# generated {seq} frames of {len(scenes)} streams in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    if args.copy_calibration_mb > 0:
        copy_calibration(args.copy_calibration_mb, dev)
    if args.tune_records and os.path.exists(args.tune_records):
        V.tune_load(args.tune_records)
    sts = [V.Stitcher(sc.rig()) for sc in scenes]
    use_surr = args.flow != "plain" and os.path.exists(args.weights)
    if use_surr:
        blob = open(args.weights, "rb").read()
        for st in sts:
            st.load_weights(blob)
            st.set_flow_mode(FLOW_MODES[args.flow], args.fb_tau)
    batch = V.Batch(sts)
    panos = [st.new_pano(dev) for st in sts]
    px = sum(st.canvas[0] * st.canvas[1] for st in sts)
    choice = [int(v) for v in sts[0].flow_variants()]
    if args.autotune:
        choice, _ = batch.autotune(frames[0], panos, reps=3)
        if args.tune_records:
            V.tune_save(args.tune_records)
    for i in range(args.warmup):
        batch.run(frames[i % seq], panos)
    torch.cuda.synchronize()
    K = args.steps
    # a serving loop bounds its queue: at most about 2 IN_FLIGHT steps enqueued
    # ahead of the GPU (a host far ahead meets the runtime's queue backpressure
    # inside graph launches, which stalls the GPU in the middle of a step).
    # Throughput: one marker event per IN_FLIGHT steps (an event recorded on the
    # stream delays the next kernel by about 5 us); latency: a second pass with
    # an event pair around every step.
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        if i % IN_FLIGHT == 0:
            if len(marks) >= 2:
                marks[-2].synchronize()
            marks.append(torch.cuda.Event())
            marks[-1].record()
        batch.run(frames[(args.warmup + i) % seq], panos)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for i in range(K):
        if i >= IN_FLIGHT:
            ends[i - IN_FLIGHT].synchronize()
        starts[i].record()
        batch.run(frames[(args.warmup + i) % seq], panos)
        ends[i].record()
    torch.cuda.synchronize()
    lat = np.array([starts[i].elapsed_time(ends[i]) for i in range(K)])
    if args.workload:
        wl = WORKLOADS[args.workload]
        streams = [f"{wl['n_cams']}x{wl['W']}x{wl['H']}" + ("_ring" if wl["ring"] else "")]
    else:
        streams = [f"{s['n_cams']}x{s['W']}x{s['H']}" for s in BATCH_STREAMS]
    out = dict(metric="panorama Mpix/s (one graph per frame step)" if args.workload else
               "panorama Mpix/s (6 uneven streams, one graph per frame step)",
               value=round(K * px / wall / 1e6, 2), unit="Mpix/s", n_gpus=1, steps=K,
               warmup=args.warmup, ms_per_step=round(wall / K * 1e3, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=args.workload or "6stream_batch", streams=streams,
                           panorama_mpix_per_step=round(px / 1e6, 3), seq_frames=seq,
                           flow_variant_per_level=choice, autotuned=bool(args.autotune),
                           pyr_tile_rows=[int(st.tuning().pyr_tile_rows) for st in sts],
                           flow=args.flow if use_surr else "plain",
                           fb_tau_px=args.fb_tau if use_surr and args.flow == "fallback" else None,
                           steps_in_flight=2 * IN_FLIGHT, parallelism="single GPU"),
               p50_ms=round(float(np.percentile(lat, 50)), 4),
               p99_ms=round(float(np.percentile(lat, 99)), 4))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
