"""Pins of the oracle's variational flow alternative (oracle/vso_var.c, the
coarse-to-fine warping scheme with brightness and gradient constancy and a
Charbonnier smoothness term): identical images give exactly zero flow; a
planted smooth displacement and a constant sub-pixel shift are recovered
(and the reverse flow is the negative); the default weights beat weights 4x
weaker and stronger against the generator's planted displacements, and beat
the plain estimator there."""
import numpy as np
from scipy.ndimage import map_coordinates

from oracle import oracle as O
from tests.test_oracle_flow import _planted, _truth_flows, texture


def test_identical_images_give_exactly_zero_flow():
    T = texture(40, 56, 3, sigma=2.0)
    f = O.var_level(T, T.copy())
    assert np.all(f == 0.0)
    assert np.all(O.var_pyramid(T, T.copy()) == 0.0)


def test_planted_smooth_displacement_is_recovered():
    h, w = 64, 96
    T, Mv, d = _planted(h, w, seed=7, amp=2.0)
    u = O.var_pyramid(T, Mv)
    inner = (slice(10, -10), slice(10, -10))
    epe = np.sqrt(((u - d) ** 2).sum(-1))[inner]
    assert epe.mean() < 0.1, epe.mean()


def test_constant_shift_and_reverse_flow():
    h, w = 64, 96
    T = texture(h, w, 8, sigma=2.0)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    s = (1.3, -0.7)
    Mv = map_coordinates(T.astype(np.float64), [ys - s[1], xs - s[0]], order=3, mode="nearest").astype(np.float32)
    fij = O.var_pyramid(T, Mv)
    fji = O.var_pyramid(Mv, T)
    inner = (slice(10, -10), slice(10, -10))
    assert np.abs(fij[inner][..., 0] - s[0]).mean() < 0.05
    assert np.abs(fij[inner][..., 1] - s[1]).mean() < 0.05
    assert np.abs(fij[inner] + fji[inner]).mean() < 0.05


def test_default_weights_against_planted_truth():
    from paper_2308_09209_amd.scenes import small_scene
    sc = small_scene(n_cams=3, W=480, H=270, overlap=0.25, ring=True, seed_config=95)
    fr = sc.frames(0)
    p0 = O.default_params()
    a0, g0 = p0.var_alpha, p0.var_gamma

    def err(**kw):
        o = O.Oracle(sc.rig(), **kw)
        o.stitch(fr)
        es = []
        for p in range(o.n_pairs):
            need = o.tap("need", p, 0).astype(bool)
            for d, t in enumerate(_truth_flows(sc, o, p)):
                es.append(np.sqrt(((o.tap("flow", p, d) - t) ** 2).sum(-1))[need])
        return float(np.concatenate(es).mean())

    e0 = err(flow=2)
    others = [err(flow=2, var_alpha=a0 / 4), err(flow=2, var_alpha=a0 * 4), err(flow=2, var_gamma=g0 / 4),
              err(flow=2, var_gamma=g0 * 4)]
    lk = err(flow=1)
    assert e0 < min(others), (e0, others)
    assert e0 < 0.3 and e0 < 0.6 * lk, (e0, lk)
