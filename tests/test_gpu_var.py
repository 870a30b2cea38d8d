"""GPU parity of the variational flow alternative (flow = 2: coarse-to-fine
warping with brightness and gradient constancy and a Charbonnier smoothness
term, lagged Jacobi steps) against the oracle's estimator of the same
reading: the plain flow context on a textured pair with a planted shift (both
directions, every level), the stitch context on small rings over several
frames (flows on the flow domain, every later step as in the default path's
parity tests), non-default weights, and one full-size 4 x 1080p frame.  The
kernels follow the oracle's FP32 operation order, so the flows are expected
bit for bit; the bar written here is the default path's (mean EPE <= 1e-3 px
per pair and direction, panorama within 1 LSB)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd import vstitch as V  # noqa: E402
from paper_2308_09209_amd.scenes import scene_for, small_scene  # noqa: E402
from tests.test_gpu_parity import check_steps, dev, lsb  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _pair(h=96, w=200, seed=3):
    from tests.test_oracle_flow import texture
    T = texture(h, w, seed, sigma=2.0)
    rng = np.random.default_rng(seed)
    M = np.roll(T, (1, 2), axis=(0, 1)) + rng.normal(size=T.shape).astype(np.float32)
    return np.round(T).astype(np.float32), np.clip(np.round(M), 0, 255).astype(np.float32)


@pytest.mark.parametrize("kw", [{}, dict(var_alpha=40.0, var_gamma=4.0, var_outer=2, var_inner=6)])
def test_plain_flow_context_matches_oracle(kw):
    T, M = _pair()
    pf = V.PlainFlow(200, 96, flow=2, **kw)
    ftm, fmt = pf(cu(T), cu(M))
    ow = dict(alpha=kw.get("var_alpha", 128.0), gamma=kw.get("var_gamma", 16.0), outer=kw.get("var_outer", 3),
              inner=kw.get("var_inner", 10))
    L = V.default_params().lk_levels
    want_tm = O.var_pyramid(T, M, levels=L, **ow)
    want_mt = O.var_pyramid(M, T, levels=L, **ow)
    for d, (g, w) in enumerate(((ftm, want_tm), (fmt, want_mt))):
        g = g.cpu().numpy()
        epe = np.sqrt(((g.astype(np.float64) - w) ** 2).sum(-1))
        say(f"[var plain {kw}] dir {d}: mean EPE {epe.mean():.2e} max {epe.max():.2e}, "
            f"identical {np.mean(np.all(g == w, -1)):.6f}")
        assert epe.mean() <= 1e-3 and epe.max() <= 1e-2
    # the planted shift is what the estimator finds in the interior
    inner = want_tm[8:-8, 8:-8]
    assert abs(np.median(inner[..., 0]) - 2.0) < 0.25 and abs(np.median(inner[..., 1]) - 1.0) < 0.25
    pf.close()


@pytest.mark.parametrize("seed,ring,n", [(96, True, 3), (41, False, 3)])
def test_stitch_with_variational_flow_matches_oracle(seed, ring, n):
    sc = small_scene(n_cams=n, W=200, H=110, overlap=0.35, ring=ring, seed_config=seed, drift=0.03)
    st = V.Stitcher(sc.rig(), debug_taps=1, flow=2)
    orc = O.Oracle(sc.rig(), flow=2)
    for t in range(3):
        frames = sc.frames(t)
        got = st.stitch(dev(frames)).cpu().numpy()
        want = orc.stitch(frames)
        d = lsb(got, want)
        say(f"[var stitch seed {seed}] frame {t}: max diff {d} LSB, identical px "
            f"{np.mean(np.all(got == want, -1)):.6f}")
        assert d <= 1
        check_steps(st, orc, f"var seed {seed} t={t}")
        np.testing.assert_array_equal(st.tap("pano_pre"), orc.tap("pano_pre"))
    st.close()


def test_variational_flow_full_size_4x1080p():
    s = scene_for("4x1920x1080_ring")
    st = V.Stitcher(s.rig(), debug_taps=1, flow=2)
    orc = O.Oracle(s.rig(), flow=2)
    frames = s.frames(0)
    got = st.stitch(dev(frames)).cpu().numpy()
    want = orc.stitch(frames)
    d = lsb(got, want)
    say(f"[var 4x1080p] max diff {d} LSB, identical px {np.mean(np.all(got == want, -1)):.6f}")
    assert d <= 1
    check_steps(st, orc, "var 4x1080p")
    st.close()
