"""Pins of the oracle's literal readings (the options that replace an adopted
reading of a passage the paper leaves open), each against values fixed by hand
or by a closed form, not by the oracle's own formulas:

* nearest-CDF histogram specification (section 2.1 step 3): small
  histograms where the nearest cumulative count, its lower tie-break and the
  inverse-CDF rule give different levels, worked out by hand;
* eq. (17) as printed: the linear-ramp frames of the meet-in-the-middle pin,
  camera i now displaced by theta_i flow_ij and camera j by theta_j flow_ji;
* eq. (4)'s overlap-only text: three cameras whose colours are camera 0's
  times planted per-channel gains; each pair's own matrix (not the chain)
  corrects camera i inside that overlap, and pixels seen by one camera keep
  their raw colour.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.rigs import T
from tests.test_oracle_blend import M_I, M_J, RAMP_I, RAMP_J, _expected_byte, _ramp


def _hist(levels_counts):
    h = np.zeros(256, np.uint32)
    for v, n in levels_counts.items():
        h[v] = n
    return h


def test_nearest_cdf_by_hand():
    # C_i: level 0 -> 2, level 1 -> 4 (then 4); C_j: level 0 -> 1, level 1 -> 4
    Gi = _hist({0: 2, 1: 2})
    Gj = _hist({0: 1, 1: 3})
    inv = O.histspec_lut(Gi, Gj)
    near = O.histspec_lut(Gi, Gj, nearest=True)
    # v = 0: C_i = 2; first w with C_j(w) >= 2 is 1; nearest is w = 0 (|1 - 2| = 1 < |4 - 2|)
    assert inv[0] == 1 and near[0] == 0
    # v = 1: C_i = 4 = C_j(1): both give 1
    assert inv[1] == 1 and near[1] == 1


def test_nearest_cdf_ties_go_to_the_lower_level():
    # C_i(0) = 3 sits halfway between C_j(0) = 2 and C_j(1) = 4
    Gi = _hist({0: 3, 5: 1})
    Gj = _hist({0: 2, 1: 2})
    assert O.histspec_lut(Gi, Gj, nearest=True)[0] == 0
    assert O.histspec_lut(Gi, Gj)[0] == 1
    # a flat stretch of C_j: C_j(w) = 2 for w = 0..6, 4 from 7; C_i(0) = 2 matches all of
    # 0..6 exactly, the smallest is 0
    Gj2 = _hist({0: 2, 7: 2})
    Gi2 = _hist({0: 2, 9: 2})
    assert O.histspec_lut(Gi2, Gj2, nearest=True)[0] == 0


def test_nearest_cdf_identity_on_equal_histograms():
    rng = np.random.default_rng(2)
    G = rng.integers(0, 50, 256).astype(np.uint32)
    lut = O.histspec_lut(G, G, nearest=True)
    occ = np.nonzero(G)[0]
    assert (lut[occ] == occ).all()


@pytest.mark.parametrize("f_ij,f_ji", [((4.0, -2.0), (-3.0, 2.5)), ((-2.5, 1.5), (2.0, -1.0))])
def test_eq17_as_printed_closed_form(f_ij, f_ji):
    W, H, off = 40, 30, 24
    Fj, (aj, bxj, byj) = _ramp(W, H, *RAMP_J)
    Fi, (ai, bxi, byi) = _ramp(W, H, *RAMP_I)
    checked = 0
    for x in range(off + 1, W - 1):
        for y in (8, 14, 21):
            dj = min(x, W - 1 - x)
            di = min(x - off, W - 1 - (x - off))
            th_i = di / (di + dj)
            th_j = 1.0 - th_i
            ui = np.clip(x - off + th_i * f_ij[0], 0, W - 1)
            vi = np.clip(y + th_i * f_ij[1], 0, H - 1)
            uj = np.clip(x + th_j * f_ji[0], 0, W - 1)
            vj = np.clip(y + th_j * f_ji[1], 0, H - 1)
            ti = np.clip((ai + bxi * ui + byi * vi) @ M_I, 0, 255)
            tj = np.clip((aj + bxj * uj + byj * vj) @ M_J, 0, 255)
            got = O.fuse_pixel(Fj, np.eye(3), M_J, x, Fi, T(-off, 0), M_I, x, y, f_ij, f_ji, literal=True)
            for c in range(3):
                assert int(got[c]) in _expected_byte(th_i * ti[c] + th_j * tj[c]), (x, y, c)
            checked += 1
    assert checked > 30


def _gain_rig():
    """three cameras, integer crops of one smooth texture (camera k at canvas
    x = 30 k), camera k's colours = the texture's times gains g_k per channel"""
    from tests.rigs import smooth_image
    W, H = 60, 24
    tex = smooth_image(H, 140, seed=21, sigma=3.0).astype(np.float64)
    tex = 40 + tex * 0.6                     # keep gains inside [0, 255]
    g = [np.array([1.0, 1.0, 1.0]), np.array([1.2, 0.9, 1.1]), np.array([0.8, 1.15, 0.95])]
    frames = [np.clip(np.round(tex[:, 30 * k:30 * k + W] * g[k]), 0, 255).astype(np.uint8) for k in range(3)]
    rig = dict(n_cams=3, W=W, H=H, H_pair=[np.eye(3), T(30, 0), T(30, 0)], H_ref=np.eye(3), ring=0,
               ring_period=0, canvas_w=120, canvas_h=H)
    return rig, frames, g


def test_overlap_only_corrects_each_overlap_with_its_own_pair_matrix():
    rig, frames, g = _gain_rig()
    lit = O.Oracle(rig, balance=0, flow=0, readings=O.READ_OVERLAP_ONLY)
    pano = lit.stitch(frames).astype(np.float64)
    # no camera is corrected as a whole
    assert np.abs(lit.tap("mk") - np.eye(3)).max() == 0
    # single-coverage columns keep the raw colours: camera 2 alone covers 90..119
    np.testing.assert_array_equal(pano[:, 90:].astype(np.uint8), frames[2][:, 30:])
    # overlap (1, 2) = columns 60..89: camera 2 corrected by the pair's own
    # matrix, which takes its colours to camera 1's (gains g1 / g2), not to
    # camera 0's; with identical geometry the fused value is then camera 1's
    # raw colour up to the rounding of the planted frames
    ov = pano[:, 62:88]
    cam1 = frames[1][:, 32:58].astype(np.float64)
    cam0_colour = cam1 / g[1]
    assert np.abs(ov - cam1).mean() < 1.0
    assert np.abs(ov - cam0_colour).mean() > 5.0
    # the default reading takes every camera to camera 0's colours instead
    dft = O.Oracle(rig, balance=0, flow=0).stitch(frames).astype(np.float64)
    assert np.abs(dft[:, 62:88] - cam0_colour).mean() < 1.0
