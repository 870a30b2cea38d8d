"""GPU: batched, graph-captured execution of several uneven streams and the
flow-kernel variants / autotuner give exactly the single-context results."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2308_09209_amd import vstitch as V  # noqa: E402
from paper_2308_09209_amd.scenes import small_scene  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(frames):
    return [torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0") for f in frames]


def scenes():
    return [small_scene(n_cams=2, W=200, H=120, overlap=0.3, drift=0.05, seed_config=91),
            small_scene(n_cams=3, W=176, H=100, overlap=0.25, ring=True, drift=0.05, seed_config=92),
            small_scene(n_cams=3, W=151, H=77, overlap=0.33, drift=0.05, seed_config=93)]


def reference(scs, n_frames):
    out = []
    for sc in scs:
        st = V.Stitcher(sc.rig())
        out.append([st.stitch(dev(sc.frames(t))).cpu().numpy() for t in range(n_frames)])
        st.close()
    return out


def test_batch_graph_replays_match_single_contexts():
    scs = scenes()
    ref = reference(scs, 4)
    sts = [V.Stitcher(sc.rig()) for sc in scs]
    b = V.Batch(sts)
    panos = [st.new_pano() for st in sts]
    scratch = torch.arange(1 << 20, device="cuda:0", dtype=torch.float32)
    for t in range(4):
        say(f"[batch] frame {t}: {len(sts)} contexts")
        frames = [dev(sc.frames(t)) for sc in scs]
        b.run(frames, panos)
        torch.cuda.synchronize()
        for c in range(len(sts)):
            np.testing.assert_array_equal(panos[c].cpu().numpy(), ref[c][t], err_msg=f"ctx {c} frame {t}")
        # eager work and a synchronisation between graph replays
        scratch.mul_(1.0001).sum().item()
    for c, st in enumerate(sts):
        assert st.state_get().frames_seen == 4
    b.close()


def test_flow_variants_are_bitwise_equal():
    sc = small_scene(n_cams=2, W=260, H=150, overlap=0.35, drift=0.05, seed_config=94)
    base = V.Stitcher(sc.rig(), debug_taps=1)
    want = [base.stitch(dev(sc.frames(t))).cpu().numpy() for t in range(2)]
    wflow = base.tap("flow", 0, 0)
    for variant in (0, 1, 2, 3, 4, 9, 10, 11, 12, 25, 26, 27, 28):
        st = V.Stitcher(sc.rig(), debug_taps=1)
        for l in range(st.info.lk_levels):
            st.set_flow_variant(l, variant)
        assert st.flow_variants() == [variant] * st.info.lk_levels
        got = [st.stitch(dev(sc.frames(t))).cpu().numpy() for t in range(2)]
        say(f"[variant {variant}] frames equal: {[bool(np.array_equal(a, b)) for a, b in zip(got, want)]}")
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(st.tap("flow", 0, 0), wflow)
        st.close()


def test_batch_autotune_keeps_results():
    scs = scenes()[:2]
    ref = reference(scs, 3)
    sts = [V.Stitcher(sc.rig()) for sc in scs]
    b = V.Batch(sts)
    panos = [st.new_pano() for st in sts]
    frames0 = [dev(sc.frames(0)) for sc in scs]
    choice, ms = b.autotune(frames0, panos, reps=2)
    say(f"[autotune] choice per level {choice}, ms {np.round(ms, 4).tolist()}")
    assert all(c in V.FLOW_VARIANT_CODES for c in choice)
    for st in sts:
        assert st.flow_variants() == choice
        assert st.state_get().frames_seen == 0
    for t in range(3):
        b.run([dev(sc.frames(t)) for sc in scs], panos)
        torch.cuda.synchronize()
        for c in range(len(sts)):
            np.testing.assert_array_equal(panos[c].cpu().numpy(), ref[c][t])
    b.close()
    V.tune_clear()   # the records of this test's rigs do not reach later tests


def test_autotune_records_apply_to_new_contexts(tmp_path):
    """vs_batch_autotune records each context's choice (flow variants and the
    fused pyramid's tile height); a context created later for the same device
    and plan shape starts from it, also after the records go through a file;
    without records it starts from the defaults.  Panoramas stay those of the
    untuned contexts."""
    scs = scenes()[:1]
    ref = reference(scs, 2)
    V.tune_clear()
    st0 = V.Stitcher(scs[0].rig())
    default = (st0.flow_variants(), st0.tuning().pyr_tile_rows)
    b = V.Batch([st0])
    panos = [st0.new_pano()]
    choice, _ = b.autotune([dev(scs[0].frames(0))], panos, reps=2)
    key = st0.tune_key()
    rec = V.tune_get(key)
    tuned = (list(rec.flow_variant)[:len(choice)], rec.pyr_tile_rows)
    say(f"[tuning records] key {key.arch.decode()} {key.canvas_w}x{key.canvas_h}: default {default}, tuned {tuned}")
    assert tuned[0] == choice and tuned[1] in (8, 16)
    assert (st0.flow_variants(), st0.tuning().pyr_tile_rows) == tuned
    b.close()
    st0.close()
    path = tmp_path / "tune.txt"
    V.tune_save(path)
    V.tune_clear()
    st1 = V.Stitcher(scs[0].rig())
    assert (st1.flow_variants(), st1.tuning().pyr_tile_rows) == default
    st1.close()
    V.tune_load(path)
    st2 = V.Stitcher(scs[0].rig())
    assert (st2.flow_variants(), st2.tuning().pyr_tile_rows) == tuned
    pano = st2.new_pano()
    for t in range(2):
        st2.stitch(dev(scs[0].frames(t)), pano=pano)
        np.testing.assert_array_equal(pano.cpu().numpy(), ref[0][t])
    st2.close()
    V.tune_clear()


def test_batch_with_mixed_pyramid_tile_heights():
    """contexts of one graph with different fused-pyramid tile heights (one
    fused launch per height) give their single-context results"""
    scs = scenes()
    ref = reference(scs, 2)
    sts = [V.Stitcher(sc.rig(), pyr_tile_rows=rows) for sc, rows in zip(scs, (16, 8, 16))]
    b = V.Batch(sts)
    panos = [st.new_pano() for st in sts]
    for t in range(2):
        b.run([dev(sc.frames(t)) for sc in scs], panos)
        torch.cuda.synchronize()
        for c in range(len(sts)):
            np.testing.assert_array_equal(panos[c].cpu().numpy(), ref[c][t], err_msg=f"ctx {c} frame {t}")
    b.close()
