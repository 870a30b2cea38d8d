"""Pins of the oracle's online colour balancing (section 2.2, eqs. (5)-(7)).

The thresholds m1, m2 (lambda = 0.05) and their 3-frame mean are fixed by
the paper; the exact shape of the piecewise curve is not (its figure is
missing), so the curve is pinned by its invariants only: parity of the curve
against the paper is unpinned."""
import math

import numpy as np

from oracle import oracle as O
from paper_2308_09209_amd.scenes import small_scene


def test_quantiles_brute_force():
    rng = np.random.default_rng(0)
    for n in [1, 7, 20, 100, 1013]:
        v = rng.integers(0, 256, n)
        h = np.bincount(v, minlength=256)
        s = np.sort(v)
        q1, q2 = O.quantiles(h, n, 5)
        # smallest level holding at least lambda (1 - lambda) of the pixels
        assert q1 == s[(5 * n + 99) // 100 - 1]
        assert q2 == s[(95 * n + 99) // 100 - 1]


def test_quantiles_constructed_histogram():
    h = np.zeros(256, np.int64)
    h[10] = 5
    h[50] = 89
    h[200] = 6
    assert O.quantiles(h, 100, 5) == (10, 200)
    h[10] = 4
    h[50] = 91
    h[200] = 5
    assert O.quantiles(h, 100, 5) == (50, 50)


def test_balance_lut_invariants():
    lam = 0.05
    t1, t2 = 255 * lam, 255 * (1 - lam)
    for m1, m2 in [(30.0, 200.0), (5.0, 250.0), (60.5, 140.25), (0.0, 255.0), (12.75, 242.25), (100, 101)]:
        lut = O.balance_lut(m1, m2).astype(int)
        assert np.all(np.diff(lut) >= 0), (m1, m2)
        assert lut[0] >= 0 and lut[255] <= 255
        s = (t2 - t1) / (m2 - m1)
        # linear part passes through (m1, t1) and (m2, t2)
        for v in range(int(math.ceil(m1)), int(math.floor(m2)) + 1):
            assert abs(lut[v] - (t1 + s * (v - m1))) <= 0.5 + 1e-9
        # continuity across the joints: the tails meet the line at m1 and m2
        for m in (m1, m2):
            lo, hi = int(math.floor(m)), int(math.ceil(m))
            if 0 < lo and hi < 255 and lo != hi:
                assert lut[hi + 1] - lut[lo - 1] <= math.ceil(3 * s) + 1


def test_balance_lut_identity_cases():
    np.testing.assert_array_equal(O.balance_lut(12.75, 242.25), np.arange(256))
    np.testing.assert_array_equal(O.balance_lut(100.0, 100.5), np.arange(256))


def test_balance_lut_gamma_tails_closed_form():
    m1, m2 = 40.0, 180.0
    t1, t2 = 12.75, 242.25
    s = (t2 - t1) / (m2 - m1)
    g1 = s * m1 / t1
    g2 = s * (255 - m2) / (255 - t2)
    lut = O.balance_lut(m1, m2)
    for v in [0, 10, 25, 39]:
        assert lut[v] == int(math.floor(t1 * (v / m1) ** g1 + 0.5))
    for v in [181, 200, 240, 255]:
        assert lut[v] == int(math.floor(255 - (255 - t2) * ((255 - v) / (255 - m2)) ** g2 + 0.5))


def test_threshold_mean_over_three_frames_and_first_frames():
    """Eqs. (6)-(7): m(T) is the mean of the thresholds of T, T-1, T-2; the
    first frame uses itself, the second the mean of the first two."""
    s = small_scene(W=120, H=72, drift=0.08)
    o = O.Oracle(s.rig())
    qs = []
    for t in range(5):
        o.stitch(s.frames(t))
        qs.append(o.tap("quant").astype(np.float64))
        mbar = o.tap("mbar")
        want = np.mean(qs[max(0, t - 2):t + 1], axis=0)
        np.testing.assert_array_equal(mbar, want)


def test_balance_applied_to_covered_pixels_only():
    s = small_scene(W=120, H=72)
    o = O.Oracle(s.rig())
    pano = o.stitch(s.frames(0))
    pre = o.tap("pano_pre")
    cov = o.tap("cover") > 0
    lut = o.tap("bal_lut")
    want = pre.copy()
    for c in range(3):
        want[..., c][cov] = lut[c][pre[..., c][cov]]
    np.testing.assert_array_equal(pano, want)
    assert np.all(pano[~cov] == 0)
    # the histogram counts covered pixels of the pre-balance panorama
    h = o.tap("pano_hist")
    for c in range(3):
        np.testing.assert_array_equal(h[c], np.bincount(pre[..., c][cov], minlength=256))
