"""Pins of the oracle's section 3.1 set-up (oracle/vso_calib.c): eqs. (8)-(12)
against a direct projection of world-plane points through the camera model
written out in numpy, eq. (14)'s revision against its closed form on points,
the Harris response and the NCC score against closed forms, and the
estimation of eq. (13)'s skew and scale parameters against a planted error
on a synthetic camera pair."""
import numpy as np

from oracle import oracle as O
from paper_2308_09209_amd.scenes import Scene


def rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def test_intrinsics_by_hand():
    K = O.calib_intrinsics(f=0.008, dx=4e-6, dy=5e-6, cx=1e-5, cy=-2e-5, u0=960.0, v0=540.0)
    np.testing.assert_allclose(K, [[2000.0, 0.0, 962.5], [0.0, 1600.0, 536.0], [0.0, 0.0, 1.0]], rtol=1e-14)


def _project(K, R, t, Xw):
    """eq. (8) written out: U = K (R x + t) / Z_c"""
    c = R @ Xw + t
    u = K @ c
    return u[:2] / u[2]


def test_plane_and_pair_homographies_against_the_camera_model():
    rng = np.random.default_rng(3)
    Ka = O.calib_intrinsics(0.006, 5e-6, 5e-6, 0.0, 0.0, 960, 540)
    Kb = O.calib_intrinsics(0.0061, 5e-6, 5.1e-6, 1e-5, 0.0, 950, 545)
    Ra, ta = rot(0.05, -0.3, 0.02), np.array([0.2, -0.1, 5.0])
    Rb, tb = rot(0.04, 0.25, -0.03), np.array([-0.3, 0.05, 5.2])
    Ha = O.calib_plane_homography(Ka, Ra, ta)
    Hb = O.calib_plane_homography(Kb, Rb, tb)
    Hab = O.calib_pair(Ha, Hb)
    for _ in range(20):
        Xw = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), 0.0])
        ua, ub = _project(Ka, Ra, ta, Xw), _project(Kb, Rb, tb, Xw)
        pa = Ha @ np.array([Xw[0], Xw[1], 1.0])
        np.testing.assert_allclose(pa[:2] / pa[2], ua, rtol=1e-12)
        q = Hab @ np.array([ub[0], ub[1], 1.0])          # camera b pixels -> camera a pixels
        np.testing.assert_allclose(q[:2] / q[2], ua, rtol=1e-10)


def test_refine_closed_form():
    H = np.array([[1.01, 0.02, 300.0], [-0.01, 0.99, 5.0], [1e-5, -2e-5, 1.0]])
    p = (3.5, -2.0, 1.02, 0.97)
    Hr = O.calib_refine(H, p)
    for (u, v) in [(10.0, 20.0), (500.0, 300.0), (1000.0, 50.0)]:
        q = H @ np.array([p[2] * u, p[3] * v, 1.0])
        want = q[:2] / q[2] + np.array(p[:2])
        r = Hr @ np.array([u, v, 1.0])
        np.testing.assert_allclose(r[:2] / r[2], want, rtol=1e-12)


def test_harris_closed_forms():
    ys, xs = np.mgrid[0:20, 0:20].astype(np.float32)
    a, b = 3.0, -2.0
    ramp = a * xs + b * ys
    # constant gradient (a, b) over the 5x5 box: Sxx = 25 a^2, Syy = 25 b^2,
    # Sxy = 25 a b, so det = 0 and R = -0.04 (25 (a^2 + b^2))^2
    assert abs(O.calib_harris(ramp, 10, 10) - (-0.04 * (25 * (a * a + b * b)) ** 2)) < 1e-3
    # a corner of two steps: positive response, larger than on either edge
    step = ((xs >= 10) & (ys >= 10)).astype(np.float32) * 100
    rc = O.calib_harris(step, 10, 10)
    assert rc > 0 and rc > O.calib_harris(step, 10, 15) and rc > O.calib_harris(step, 15, 10)


def test_ncc_closed_forms():
    rng = np.random.default_rng(4)
    A = rng.uniform(0, 255, (30, 30)).astype(np.float32)
    assert abs(O.calib_ncc(A, 12, 12, 2 * A + 3, 12, 12) - 1.0) < 1e-5
    assert abs(O.calib_ncc(A, 12, 12, -A + 255, 12, 12) + 1.0) < 1e-5
    assert O.calib_ncc(A, 12, 12, np.full_like(A, 7.0), 12, 12) == 0.0
    shifted = np.roll(A, (1, -2), axis=(0, 1))
    assert abs(O.calib_ncc(A, 12, 12, shifted, 10, 13) - 1.0) < 1e-6


def _pair_scene():
    sc = Scene(n_cams=2, W=320, H=200, overlap=0.45, ring=False, tex_h=240, resid=0.0, colour=False, config=97)
    rig = sc.rig()
    return sc, np.asarray(rig["H_pair"][1])      # camera 1 pixels -> camera 0 pixels


def _reproj(Ha, Hb, pts):
    out = []
    for (u, v) in pts:
        p, q = Ha @ [u, v, 1.0], Hb @ [u, v, 1.0]
        out.append(np.hypot(*(p[:2] / p[2] - q[:2] / q[2])))
    return float(np.mean(out))


import pytest


@pytest.mark.parametrize("err,radius", [((2.6, -1.8, 1.012, 0.99), 6), ((-3.5, 2.2, 0.985, 1.015), 8)])
def test_estimate_recovers_a_planted_skew_and_scale_error(err, radius):
    sc, H_true = _pair_scene()
    frames = sc.frames(0)
    # the coarse calibration is off by a skew and a scale (eq. (13)'s parameters)
    H_given = O.calib_refine(H_true, err)
    pts = [(u, v) for u in range(20, 140, 20) for v in range(20, 180, 20)]
    before = _reproj(H_given, H_true, pts)
    p, nm, ni = O.calib_estimate(frames[1], frames[0], H_given, margin=16, radius=radius)
    assert p is not None and ni >= 10, (nm, ni)
    after = _reproj(O.calib_refine(H_given, p), H_true, pts)
    assert before > 2.0 and after < 0.25, (before, after, p, nm, ni)
