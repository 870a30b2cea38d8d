"""GPU: the learned flow surrogate inside the frame, through the C ABI,
against the oracle on the same seeded inputs and seeded network weights.

Bars.  The network's sums run on the matrix cores in FP32 and the oracle's in
exact FP64, so a hidden activation that sits on a BF16 rounding boundary can
round the other way (one BF16 step, 2^-8 relative): the level-2 prediction is
held to 1e-3 relative L2, the level-0 flow to 1e-3 px mean EPE (the plain
flow's bar), the fixed-point forward-backward sums to 1 % plus one unit per
pixel.  The panorama reads the flow through a bilinear resample of bytes (at
most 255 levels per px), the colour matrix (at most its largest absolute
column sum) and the balancing LUT (at most its largest step), so a flow that
differs by d px can move a pixel by ceil(step * (ceil(255 * g * d) + 1))
levels: the panorama is held to that bound, computed from the measured flow
difference, and to 1 LSB on all but 1e-3 of its pixels.  Where the two sides
run identical arithmetic the result must be bit-equal: threshold 0 reproduces
the plain path, an unlimited threshold reproduces the surrogate-only path, a
zero network reproduces the zero-flow path, and a bias-only network gives its
closed form.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd import scenes as S  # noqa: E402
from paper_2308_09209_amd import vstitch as V  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(frames):
    return [torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0") for f in frames]


def lsb(a, b):
    return int(np.abs(a.astype(np.int64) - b.astype(np.int64)).max()) if a.size else 0


def rel_l2(a, b):
    return float(np.linalg.norm(a.astype(np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture(scope="module")
def ring():
    return S.small_scene(n_cams=3, W=200, H=120, overlap=0.35, ring=True, seed_config=92)


@pytest.fixture(scope="module")
def blob():
    ws, bs = S.random_net(11)
    return S.nn_blob(ws, bs)


def gpu_run(scene, n, blob=None, mode=V.FLOW_PLAIN, tau=0.0, **params):
    st = V.Stitcher(scene.rig(), **params)
    if blob is not None:
        st.load_weights(blob)
    if mode != V.FLOW_PLAIN:
        st.set_flow_mode(mode, tau)
    panos, infos = [], []
    for t in range(n):
        pano, _, info = st.stitch(dev(scene.frames(t)), want_info=True)
        panos.append(pano.cpu().numpy())
        infos.append(info)
    return st, panos, infos


def check_pano(st, orc, got, want, dmax, label):
    """got vs want within the bound that a flow difference of dmax px allows"""
    diff = np.abs(got.astype(np.int64) - want.astype(np.int64))
    g = float(np.abs(orc.tap("mk")).sum(axis=1).max())
    lut = orc.tap("bal_lut").astype(np.int64)
    step = max(1, int(np.abs(np.diff(lut, axis=1)).max()))
    bound = int(np.ceil(step * (np.ceil(255.0 * g * dmax) + 1)))
    frac = float((diff > 1).mean())
    say(f"  {label}: panorama max |diff| {int(diff.max())} LSB (bound {bound}), {frac:.2e} of pixels above 1 LSB")
    assert diff.max() <= bound and frac <= 1e-3, (label, int(diff.max()), bound, frac)


def check_pre(st, orc, dmax, label):
    """the pre-balance panorama (needs debug_taps) within the bound a flow
    difference of dmax px allows before the balancing LUT: ceil(255 g dmax) + 1
    levels, and 1 LSB on all but 1e-3 of its pixels"""
    diff = np.abs(st.tap("pano_pre").astype(np.int64) - orc.tap("pano_pre").astype(np.int64))
    g = float(np.abs(orc.tap("mk")).sum(axis=1).max())
    bound = int(np.ceil(255.0 * g * dmax)) + 1
    frac = float((diff > 1).mean())
    say(f"  {label}: pre-balance max |diff| {int(diff.max())} LSB (bound {bound}), {frac:.2e} of pixels above 1 LSB")
    assert diff.max() <= bound and frac <= 1e-3, (label, int(diff.max()), bound, frac)


def check_vs_oracle(st, orc, label):
    """per-step checks; returns the largest level-0 flow difference (px)"""
    dmax = 0.0
    for p in range(orc.n_pairs):
        for d in (0, 1):
            a, b = st.tap("surr_pred", p, d), orc.tap("surr_pred", p, d)
            e = rel_l2(a, b)
            assert e <= 1e-3, (label, p, d, e)
            fa, fb = st.tap("flow", p, d), orc.tap("flow", p, d)
            epe = np.sqrt(((fa.astype(np.float64) - fb) ** 2).sum(-1))
            assert epe.mean() <= 1e-3, (label, p, d, epe.mean(), epe.max())
            dmax = max(dmax, float(epe.max()))
            if e > 0 or epe.max() > 0:
                say(f"  {label} pair {p} dir {d}: prediction rel L2 {e:.2e}, flow EPE mean {epe.mean():.2e} "
                    f"max {epe.max():.2e}")
        (sg, ng), (so, no) = st.tap("fb")[p], orc.tap("fb")[p]
        assert ng == no, (label, p)
        assert abs(int(sg) - int(so)) <= 0.01 * int(so) + int(no), (label, p, sg, so)
    np.testing.assert_array_equal(st.tap("surr_ok"), orc.tap("surr_ok"))
    return dmax


@pytest.mark.parametrize("mode", [V.FLOW_SURROGATE, V.FLOW_SURROGATE_FALLBACK])
def test_surrogate_frames_match_oracle(ring, blob, mode):
    tau = 1e6 if mode == V.FLOW_SURROGATE_FALLBACK else 0.0
    st = V.Stitcher(ring.rig(), debug_taps=1)
    st.load_weights(blob)
    st.set_flow_mode(mode, tau)
    orc = O.Oracle(ring.rig())
    orc.set_surrogate(blob, mode, tau)
    for t in range(3):
        say(f"[surrogate mode {mode}] frame {t}")
        pano, _, info = st.stitch(dev(ring.frames(t)), want_info=True)
        want = orc.stitch(ring.frames(t))
        dmax = check_vs_oracle(st, orc, f"mode {mode} frame {t}")
        np.testing.assert_array_equal(st.tap("quant"), orc.tap("quant"))
        check_pre(st, orc, dmax, f"mode {mode} frame {t}")
        check_pano(st, orc, pano.cpu().numpy(), want, dmax, f"mode {mode} frame {t}")
        fb = orc.tap("fb")
        for p in range(orc.n_pairs):
            assert info.surr_ok[p] == 1
            assert abs(info.fb_err[p] - fb[p][0] / 256.0 / fb[p][1]) <= 0.01 * info.fb_err[p] + 1 / 256


def test_zero_threshold_is_the_plain_path_bit_for_bit(ring, blob):
    _, plain, _ = gpu_run(ring, 3)
    st, surr, infos = gpu_run(ring, 3, blob, V.FLOW_SURROGATE_FALLBACK, 0.0)
    for a, b in zip(plain, surr):
        assert np.array_equal(a, b)
    assert np.all(st.tap("surr_ok") == 0)
    assert all(infos[-1].surr_ok[p] == 0 and infos[-1].fb_err[p] >= 0 for p in range(st.n_pairs))


def test_unlimited_threshold_is_the_surrogate_path_bit_for_bit(ring, blob):
    _, a, _ = gpu_run(ring, 2, blob, V.FLOW_SURROGATE)
    _, b, _ = gpu_run(ring, 2, blob, V.FLOW_SURROGATE_FALLBACK, 1e6)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_mixed_fallback_decisions_match_oracle(ring, blob):
    orc = O.Oracle(ring.rig())
    orc.set_surrogate(blob, O.FLOW_SURROGATE)
    orc.stitch(ring.frames(0))
    fb = orc.tap("fb").astype(np.float64)
    err = np.sort(fb[:, 0] / fb[:, 1] / 256.0)
    gaps = err[1:] / err[:-1]
    k = int(np.argmax(gaps))
    if gaps[k] < 1.05:
        pytest.skip(f"pair errors too close to split: {err}")
    tau = float(np.sqrt(err[k] * err[k + 1]))
    say(f"[mixed] pair errors {np.round(err, 4)} px, threshold {tau:.4f}")
    st, panos, _ = gpu_run(ring, 1, blob, V.FLOW_SURROGATE_FALLBACK, tau)
    o2 = O.Oracle(ring.rig())
    o2.set_surrogate(blob, O.FLOW_FALLBACK, tau)
    want = o2.stitch(ring.frames(0))
    ok = o2.tap("surr_ok")
    assert 0 < ok.sum() < len(ok)
    dmax = check_vs_oracle(st, o2, "mixed")
    check_pano(st, o2, panos[0], want, dmax, "mixed")


def test_zero_network_is_the_zero_flow_path(ring):
    layers = S.SURROGATE_LAYERS
    zero = S.nn_blob([np.zeros((co, 9, ci)) for ci, co in layers], [np.zeros(co) for _, co in layers])
    _, a, _ = gpu_run(ring, 2, flow=0)
    _, b, _ = gpu_run(ring, 2, zero, V.FLOW_SURROGATE)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_bias_only_network_closed_form(ring):
    layers = S.SURROGATE_LAYERS
    ws = [np.zeros((co, 9, ci)) for ci, co in layers]
    bs = [np.zeros(co) for _, co in layers]
    bs[-1][0] = 0.25
    st, _, _ = gpu_run(ring, 1, S.nn_blob(ws, bs), V.FLOW_SURROGATE)
    for p in range(st.n_pairs):
        need = st.tap("need", p, 0).astype(bool)
        for d in (0, 1):
            f = st.tap("flow", p, d)
            assert np.all(f[need] == np.float32([1.0, 0.0])) and np.all(f[~need] == 0)
        s, n = st.tap("fb")[p]
        assert n == need.sum() and s == 512 * n


def test_batch_with_surrogate_and_recapture(blob):
    scs = [S.small_scene(n_cams=3, W=200, H=120, overlap=0.35, ring=True, seed_config=93),
           S.small_scene(n_cams=2, W=160, H=96, overlap=0.3, seed_config=94)]
    ref = []
    for i, sc in enumerate(scs):
        mode = V.FLOW_SURROGATE if i == 0 else V.FLOW_PLAIN
        _, panos, _ = gpu_run(sc, 2, blob if i == 0 else None, mode)
        ref.append(panos)
    sts = [V.Stitcher(sc.rig()) for sc in scs]
    sts[0].load_weights(blob)
    sts[0].set_flow_mode(V.FLOW_SURROGATE)
    b = V.Batch(sts)
    panos = [st.new_pano() for st in sts]
    for t in range(2):
        b.run([dev(sc.frames(t)) for sc in scs], panos)
        torch.cuda.synchronize()
        for i in range(2):
            assert np.array_equal(panos[i].cpu().numpy(), ref[i][t]), (t, i)
    # a mode change after capture makes the batch recapture: the same switch
    # on a single context gives the same frame
    one = V.Stitcher(scs[0].rig())
    one.load_weights(blob)
    one.set_flow_mode(V.FLOW_SURROGATE)
    for t in range(2):
        one.stitch(dev(scs[0].frames(t)))
    one.set_flow_mode(V.FLOW_SURROGATE_FALLBACK, 0.0)
    want = one.stitch(dev(scs[0].frames(2))).cpu().numpy()
    sts[0].set_flow_mode(V.FLOW_SURROGATE_FALLBACK, 0.0)
    b.run([dev(sc.frames(2)) for sc in scs], panos)
    torch.cuda.synchronize()
    assert np.array_equal(panos[0].cpu().numpy(), want)
    assert np.all(sts[0].tap("surr_ok") == 0)


def test_surrogate_full_size_ring_frame_matches_oracle(blob):
    sc = S.scene_for("4x1920x1080_ring")
    st = V.Stitcher(sc.rig(), debug_taps=1)
    st.load_weights(blob)
    st.set_flow_mode(V.FLOW_SURROGATE)
    orc = O.Oracle(sc.rig())
    orc.set_surrogate(blob, O.FLOW_SURROGATE)
    say("[4x1920x1080 ring, surrogate] frame 0")
    pano = st.stitch(dev(sc.frames(0)))
    torch.cuda.synchronize()
    want = orc.stitch(sc.frames(0))
    dmax = check_vs_oracle(st, orc, "4x1080p")
    check_pre(st, orc, dmax, "4x1080p")
    check_pano(st, orc, pano.cpu().numpy(), want, dmax, "4x1080p")


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2308_09209_amd",
                       "weights", "flow_surrogate.vsnn")


def test_trained_surrogate_gain_on_the_4x1080p_ring():
    """What the trained network gains over the method without it, inside the
    4 x 1920x1080 ring: flows within 0.5 px mean end-point error of the plain
    estimator's over the overlaps, in less device time per frame."""
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained surrogate weights in the tree")
    blob = open(WEIGHTS, "rb").read()
    sc = S.scene_for("4x1920x1080_ring")
    frames = [dev(sc.frames(t)) for t in range(4)]
    plain = V.Stitcher(sc.rig())
    surr = V.Stitcher(sc.rig())
    surr.load_weights(blob)
    surr.set_flow_mode(V.FLOW_SURROGATE)
    errs = []
    for t in range(3):
        plain.stitch(frames[t])
        surr.stitch(frames[t])
        torch.cuda.synchronize()
        for p in range(plain.n_pairs):
            need = plain.tap("need", p, 0).astype(bool)
            for d in (0, 1):
                a, b = surr.tap("flow", p, d), plain.tap("flow", p, d)
                errs.append(np.sqrt(((a.astype(np.float64) - b) ** 2).sum(-1))[need])
    e = np.concatenate(errs)
    times = {}
    for name, st in (("plain", plain), ("surrogate", surr)):
        st.set_timing(True)
        for i in range(20):
            st.stitch(frames[i % 4])
        ms, n = st.timing()
        st.set_timing(False)
        times[name] = ms / n
    say(f"[gain] EPE vs plain: mean {e.mean():.4f} px, p99 {np.percentile(e, 99):.4f} px; frame "
        f"{times['plain'][5]:.4f} ms plain, {times['surrogate'][5]:.4f} ms surrogate "
        f"(flow step {times['plain'][2]:.4f} -> {times['surrogate'][2]:.4f} ms)")
    assert e.mean() <= 0.5
    assert times["surrogate"][5] < times["plain"][5]


def test_batch_of_surrogate_contexts_runs_their_chains_side_by_side(blob):
    """Three contexts with the surrogate in one graph: their network chains are
    captured as parallel branches; every replay equals the single contexts."""
    scs = [S.small_scene(n_cams=3, W=200, H=120, overlap=0.35, ring=True, seed_config=98),
           S.small_scene(n_cams=2, W=160, H=96, overlap=0.3, seed_config=99),
           S.small_scene(n_cams=4, W=180, H=100, overlap=0.3, seed_config=100)]
    modes = [(V.FLOW_SURROGATE, 0.0), (V.FLOW_SURROGATE_FALLBACK, 0.0), (V.FLOW_SURROGATE_FALLBACK, 1e6)]
    ref = [gpu_run(sc, 3, blob, m, tau)[1] for sc, (m, tau) in zip(scs, modes)]
    sts = []
    for sc, (m, tau) in zip(scs, modes):
        st = V.Stitcher(sc.rig())
        st.load_weights(blob)
        st.set_flow_mode(m, tau)
        sts.append(st)
    b = V.Batch(sts)
    panos = [st.new_pano() for st in sts]
    for t in range(3):
        b.run([dev(sc.frames(t)) for sc in scs], panos)
        torch.cuda.synchronize()
        for i in range(3):
            assert np.array_equal(panos[i].cpu().numpy(), ref[i][t]), (t, i)
