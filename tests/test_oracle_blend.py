"""Pins of the oracle's fusion (eqs. (16)-(18)), its flow-input luma and its
colour chain (eq. (4) across cameras), each against a value fixed from
outside the oracle's own formulas:

* eq. (16): two flat-colour cameras at an integer offset; the overlap columns
  must blend from camera j's colour at camera i's border to camera i's colour
  at camera j's border, with weights taken from the crop geometry by hand;
* eq. (17): frames that are linear ramps (bilinear resampling reproduces them)
  and a given constant flow pair; the fused value has a closed form in
  float64 for the meet-in-the-middle displacement;
* the luma: the BT.601 weights (0.299, 0.587, 0.114) on grey and pure
  primaries, end to end through the flow-input pyramid;
* the chain: planted non-commuting colour matrices per camera; every camera's
  composed matrix must take its colours to camera 0's (a matrix inverse
  computed by numpy, not a composition).
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.rigs import T


def _expected_byte(v):
    """Accept the float64 closed form's rounding; at a near-tie either side."""
    v = min(max(v, 0.0), 255.0)
    lo = int(np.floor(v + 0.5))
    if abs((v - np.floor(v)) - 0.5) < 1e-3:
        return {int(np.floor(v)), int(np.floor(v)) + 1}
    return {lo}


def _flat_pair(A, B, W=40, H=12, off=24):
    fj = np.empty((H, W, 3), np.uint8)
    fj[:] = A
    fi = np.empty((H, W, 3), np.uint8)
    fi[:] = B
    rig = dict(n_cams=2, W=W, H=H, H_pair=[np.eye(3), T(off, 0)], H_ref=np.eye(3), ring=0,
               ring_period=0, canvas_w=off + W, canvas_h=H)
    return rig, [fj, fi]


def test_eq16_weights_follow_each_cameras_own_border():
    # camera j covers canvas columns 0..39, camera i columns 24..63; in the
    # overlap 24..39 the distance to camera j's vertical border is
    # min(x, 39 - x), to camera i's min(x - 24, 63 - x); camera i's weight is
    # its distance over the sum, so the overlap runs from j's colour at
    # x = 24 (i's border) to i's colour at x = 39 (j's border)
    A = np.array([40, 100, 220])
    B = np.array([200, 30, 90])
    W, off = 40, 24
    rig, frames = _flat_pair(A, B, W=W, off=off)
    orc = O.Oracle(rig, color_window=0, balance=0, flow=0)
    pano = orc.stitch(frames)
    assert (pano[:, :off] == A).all() and (pano[:, W:] == B).all()
    for x in range(off, W):
        dj = min(x, W - 1 - x)
        di = min(x - off, W - 1 - (x - off))
        th_i = di / (di + dj)
        for c in range(3):
            want = _expected_byte(A[c] + th_i * (B[c] - A[c]))
            got = set(int(v) for v in pano[:, x, c])
            assert got <= want, (x, c, got, want)
    assert (pano[:, off] == A).all() and (pano[:, W - 1] == B).all()


def test_eq16_end_to_end_with_flows_estimated_on_flat_views():
    # the plain estimator on flat views has no gradient, so its flows are 0
    # and the blend is the same as with the flow switched off
    rig, frames = _flat_pair(np.array([10, 250, 128]), np.array([250, 10, 64]))
    a = O.Oracle(rig, color_window=0, balance=0, flow=0).stitch(frames)
    b = O.Oracle(rig, color_window=0, balance=0, flow=1).stitch(frames)
    assert (a == b).all()


def _ramp(W, H, a, bx, by):
    ys, xs = np.mgrid[0:H, 0:W]
    out = np.stack([a[c] + bx[c] * xs + by[c] * ys for c in range(3)], -1)
    assert out.min() >= 0 and out.max() <= 255
    return out.astype(np.uint8), (np.asarray(a, float), np.asarray(bx, float), np.asarray(by, float))


RAMP_J = ([20, 200, 10], [3, -2, 1], [2, 1, 5])
RAMP_I = ([50, 100, 240], [2, 3, -4], [3, -1, -1])
M_J = np.array([[1.05, 0.02, 0.0], [0.0, 0.95, 0.03], [0.01, 0.0, 1.1]])
M_I = np.array([[0.9, 0.05, 0.0], [0.02, 1.1, -0.03], [0.0, 0.04, 0.95]])


@pytest.mark.parametrize("f_ij,f_ji", [((4.0, -2.0), (-3.0, 2.5)), ((-2.5, 1.5), (2.0, -1.0)),
                                       ((0.0, 0.0), (0.0, 0.0))])
def test_eq17_meet_in_the_middle_closed_form(f_ij, f_ji):
    # camera j = canvas coordinates, camera i = canvas shifted by 24 px; both
    # frames are linear ramps, so a bilinear sample at any point of the frame
    # is the ramp's value there.  Camera i is read at x + theta_j f_ij and camera
    # j at x + theta_i f_ji; colours are row vectors times M.
    W, H, off = 40, 30, 24
    Fj, (aj, bxj, byj) = _ramp(W, H, *RAMP_J)
    Fi, (ai, bxi, byi) = _ramp(W, H, *RAMP_I)
    hj = np.eye(3)
    hi = T(-off, 0)
    checked = 0
    for x in range(off + 1, W - 1):
        for y in (8, 14, 21):
            dj = min(x, W - 1 - x)
            di = min(x - off, W - 1 - (x - off))
            th_i = di / (di + dj)
            th_j = 1.0 - th_i
            # positions outside a frame clamp to its border (the sampler's rule)
            ui = np.clip(x - off + th_j * f_ij[0], 0, W - 1)
            vi = np.clip(y + th_j * f_ij[1], 0, H - 1)
            uj = np.clip(x + th_i * f_ji[0], 0, W - 1)
            vj = np.clip(y + th_i * f_ji[1], 0, H - 1)
            si = ai + bxi * ui + byi * vi
            sj = aj + bxj * uj + byj * vj
            ti = np.clip(si @ M_I, 0, 255)
            tj = np.clip(sj @ M_J, 0, 255)
            got = O.fuse_pixel(Fj, hj, M_J, x, Fi, hi, M_I, x, y, f_ij, f_ji)
            for c in range(3):
                assert int(got[c]) in _expected_byte(th_i * ti[c] + th_j * tj[c]), (x, y, c)
            checked += 1
    assert checked > 30


def test_eq17_literal_reading_would_differ():
    # guard on the fixture: moving camera i by theta_i f_ij (the equation as
    # printed) instead of theta_j f_ij gives other bytes at this pixel, so the
    # closed-form test above can tell the two readings apart
    W, H, off, x, y = 40, 30, 24, 26, 14
    _, (ai, bxi, byi) = _ramp(W, H, *RAMP_I)
    _, (aj, bxj, byj) = _ramp(W, H, *RAMP_J)
    f_ij, f_ji = (4.0, -2.0), (-3.0, 2.5)
    dj, di = min(x, W - 1 - x), min(x - off, W - 1 - (x - off))
    th_i = di / (di + dj)
    th_j = 1 - th_i

    def fused(wi, wj):
        si = ai + bxi * (x - off + wi * f_ij[0]) + byi * (y + wi * f_ij[1])
        sj = aj + bxj * (x + wj * f_ji[0]) + byj * (y + wj * f_ji[1])
        return th_i * (si @ M_I) + th_j * (sj @ M_J)

    assert np.abs(np.floor(fused(th_j, th_i) + 0.5) - np.floor(fused(th_i, th_j) + 0.5)).max() >= 2


def test_luma_bt601_weights():
    for v in (0, 1, 77, 128, 254, 255):
        assert O.luma(v, v, v) == v                       # grey keeps its level
    for v in range(0, 256, 5):
        assert abs(O.luma(v, 0, 0) - 0.299 * v) <= 1.0
        assert abs(O.luma(0, v, 0) - 0.587 * v) <= 1.0
        assert abs(O.luma(0, 0, v) - 0.114 * v) <= 1.0


def test_luma_channel_order_end_to_end():
    # camera j pure red, camera i pure blue: the flow input of the strips is
    # their BT.601 luma (RGB byte order), level 0 of the pyramid
    rig, frames = _flat_pair(np.array([200, 0, 0]), np.array([0, 0, 200]))
    orc = O.Oracle(rig, color_window=0, balance=0)
    orc.stitch(frames)
    yj = orc.tap("pyr", 0, 0 * 8 + 0)
    yi = orc.tap("pyr", 0, 1 * 8 + 0)
    assert abs(float(yj.mean()) - 0.299 * 200) <= 1.0 and yj.min() == yj.max()
    assert abs(float(yi.mean()) - 0.114 * 200) <= 1.0 and yi.min() == yi.max()


def test_chain_recovers_planted_non_commuting_matrices():
    # camera k's colours are camera 0's times P_k (row vectors), P_0 = I; the
    # pair (k-1, k) matrix takes camera k's colours to camera k-1's:
    # inv(P_k) P_(k-1).  Each camera's chained matrix must then be inv(P_k).
    rng = np.random.default_rng(11)
    P = [np.eye(3)]
    for _ in range(4):
        P.append(np.eye(3) + rng.uniform(-0.2, 0.2, (3, 3)))
    assert np.abs(P[1] @ P[2] - P[2] @ P[1]).max() > 1e-2      # they do not commute
    Mpair = [np.linalg.inv(P[k]) @ P[k - 1] for k in range(1, len(P))]
    Mk = O.chain_colour(Mpair)
    for k in range(len(P)):
        assert np.abs(Mk[k] - np.linalg.inv(P[k])).max() <= 1e-12, k
