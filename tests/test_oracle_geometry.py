"""Pins of the oracle's geometry: rounding, homography apply, bilinear
resampling, the plan (overlap strips) and the end-to-end planted truths.

Section 3.1 (pre-warp) and section 2.1 step 1 (overlap from the homography);
eqs. (15)-(18) for the blend of identical views.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.rigs import crop_rig, smooth_image, T


def test_round8_half_up_and_clamp():
    assert O.round8(0.5) == 1
    assert O.round8(2.5) == 3
    assert O.round8(1.4999) == 1
    assert O.round8(-3.0) == 0
    assert O.round8(255.49) == 255
    assert O.round8(400.0) == 255


def test_homography_identity_and_validity():
    h = np.eye(3, dtype=np.float32)
    ok, u, v = O.hom_valid(h, 5.0, 7.0, 10, 10)
    assert ok and u == 5.0 and v == 7.0
    assert not O.hom_valid(h, 9.5, 0.0, 10, 10)[0]      # beyond W-1
    assert O.hom_valid(h, 9.0, 9.0, 10, 10)[0]          # exactly W-1, H-1 is inside
    assert not O.hom_valid(h, -0.001, 0.0, 10, 10)[0]
    neg = np.diag([1.0, 1.0, -1.0]).astype(np.float32)  # w <= 0: invalid, position (0, 0)
    ok, u, v = O.hom_valid(neg, 3.0, 3.0, 10, 10)
    assert not ok and u == 0.0 and v == 0.0


def test_homography_projective_closed_form():
    # a projective map with dyadic coefficients is evaluated exactly in FP32
    h = np.array([[0.5, 0.25, 3.0], [0.125, 0.75, -2.0], [0.0, 0.0, 2.0]], np.float32)
    ok, u, v = O.hom_valid(h, 8.0, 4.0, 100, 100)
    assert ok and u == (0.5 * 8 + 0.25 * 4 + 3) / 2 and v == (0.125 * 8 + 0.75 * 4 - 2) / 2


def test_bilinear_integer_positions_are_exact():
    img = smooth_image(9, 11, seed=3)
    for (x, y) in [(0, 0), (10, 8), (4, 5), (10, 0)]:
        for c in range(3):
            assert O.bilinear(img, c, float(x), float(y)) == float(img[y, x, c])


def test_bilinear_half_pixel_is_mean_of_two_taps():
    img = smooth_image(9, 11, seed=4)
    for c in range(3):
        r = O.bilinear(img, c, 3.5, 2.0)
        assert r == (float(img[2, 3, c]) + float(img[2, 4, c])) / 2
        assert O.round8(r) == int(np.floor((int(img[2, 3, c]) + int(img[2, 4, c])) / 2 + 0.5))


def test_bilinear_reproduces_bilinear_function():
    # f = 3 + 2x + 5y + xy is reproduced exactly at dyadic positions
    ys, xs = np.mgrid[0:6, 0:7]
    f = 3 + 2 * xs + 5 * ys + xs * ys
    img = np.repeat(f[..., None], 3, axis=2).astype(np.uint8)
    for (u, v) in [(1.25, 2.5), (4.75, 0.125), (5.5, 4.5)]:
        assert O.bilinear(img, 1, u, v) == 3 + 2 * u + 5 * v + u * v


def test_bilinear_clamps_outside():
    img = smooth_image(5, 6, seed=5)
    assert O.bilinear(img, 0, -3.0, -7.0) == img[0, 0, 0]
    assert O.bilinear(img, 2, 99.0, 99.0) == img[4, 5, 2]
    assert O.bilinear(img, 1, 2.0, -0.5) == img[0, 2, 1]


def test_plan_chain_strip_is_the_overlap():
    tex = smooth_image(40, 200, seed=1)
    rig, frames = crop_rig(tex, 100, 40, [(0, 0), (70, 0)])
    o = O.Oracle(rig)
    assert o.n_pairs == 1
    assert o.strip_box(0) == (70, 0, 30, 40)
    assert o.plan.n_covered == 170 * 40


def test_plan_ring_closure_pair_wraps():
    tex = smooth_image(30, 240, seed=2, periodic_x=True)
    rig, frames = crop_rig(tex, 100, 30, [(0, 0), (80, 0), (160, 0)], ring_period=240)
    o = O.Oracle(rig)
    assert o.n_pairs == 3
    assert o.strip_box(0) == (80, 0, 20, 30)
    assert o.strip_box(1) == (160, 0, 20, 30)
    # closure pair (2, 0): camera 0 one period to the right
    assert o.strip_box(2) == (240, 0, 20, 30)
    assert (o.plan.pair_j[2], o.plan.pair_i[2], o.plan.pair_si[2]) == (2, 0, 1)
    assert o.plan.n_covered == 240 * 30


def test_plan_rejects_triple_overlap_and_gaps():
    tex = smooth_image(20, 300, seed=3)
    rig, _ = crop_rig(tex, 100, 20, [(0, 0), (40, 0), (80, 0)])   # x in [80,100) covered 3x
    with pytest.raises(O.OracleError, match="-2"):
        O.Oracle(rig)
    rig, _ = crop_rig(tex, 100, 20, [(0, 0), (150, 0)])           # no overlap
    with pytest.raises(O.OracleError, match="-2"):
        O.Oracle(rig)


def test_plan_rejects_singular_homography():
    tex = smooth_image(20, 300, seed=3)
    rig, _ = crop_rig(tex, 100, 20, [(0, 0), (60, 0)])
    rig["H_pair"][1] = np.zeros((3, 3))
    with pytest.raises(O.OracleError, match="-1"):
        O.Oracle(rig)


@pytest.mark.parametrize("flow", [0, 1])
def test_identity_views_reproduce_the_texture(flow):
    """Integer-crop cameras of one texture, identical colours, balance off:
    the panorama is the texture itself, bit for bit (identity pre-warp,
    integer shift, flow exactly zero, M = I, theta_i + theta_j = 1)."""
    tex = smooth_image(48, 230, seed=11)
    rig, frames = crop_rig(tex, 96, 48, [(0, 0), (67, 0), (134, 0)])
    o = O.Oracle(rig, balance=0, flow=flow)
    pano = o.stitch(frames)
    np.testing.assert_array_equal(pano, tex)
    assert np.all(o.tap("flow", 0, 0) == 0) and np.all(o.tap("flow", 1, 1) == 0)
    assert np.all(o.tap("flags") == 0)


def test_identity_views_ring_wraps_exactly():
    tex = smooth_image(40, 216, seed=12, periodic_x=True)
    rig, frames = crop_rig(tex, 90, 40, [(0, 0), (72, 0), (144, 0)], ring_period=216)
    o = O.Oracle(rig, balance=0)
    pano = o.stitch(frames)
    np.testing.assert_array_equal(pano, tex)


def test_flipped_camera_is_an_exact_permutation():
    tex = smooth_image(40, 160, seed=13)
    rig, frames = crop_rig(tex, 100, 40, [(0, 0), (60, 0)])
    # camera 1 mounted upside down: its frame is rotated by 180 degrees
    frames[1] = np.ascontiguousarray(frames[1][::-1, ::-1])
    flip = np.array([[-1.0, 0, 99.0], [0, -1.0, 39.0], [0, 0, 1.0]])
    Hk1 = T(60, 0) @ flip
    rig["H_pair"][1] = np.linalg.inv(rig["H_ref"]) @ Hk1
    o = O.Oracle(rig, balance=0)
    pano = o.stitch(frames)
    np.testing.assert_array_equal(pano, tex)


def test_half_pixel_translation_is_mean_of_taps():
    """A camera shifted by half a pixel: its single-coverage region is the
    round-half-up mean of two horizontally adjacent texture pixels."""
    tex = smooth_image(30, 200, seed=14)
    rig, frames = crop_rig(tex, 100, 30, [(0, 0), (60, 0)])
    # camera 1 shows the texture from x = 60 on, but is declared at 59.5
    rig["H_pair"][1] = T(59.5, 0)
    o = O.Oracle(rig, balance=0, flow=0, color_window=0)
    pano = o.stitch(frames)
    # canvas x in (100, 159): only camera 1 covers it; camera u = x - 59.5
    xs = np.arange(101, 159)
    u0 = (xs - 60)  # floor(x - 59.5) = x - 60 -> taps frames[1][:, u0] and u0 + 1
    a = frames[1][:, u0].astype(int)
    b = frames[1][:, u0 + 1].astype(int)
    np.testing.assert_array_equal(pano[:, xs], np.floor((a + b) / 2 + 0.5).astype(np.uint8))


def test_deterministic():
    tex = smooth_image(40, 160, seed=15)
    rig, frames = crop_rig(tex, 100, 40, [(0, 0), (60, 0)])
    frames[1] = np.clip(frames[1].astype(int) * 1.1, 0, 255).astype(np.uint8)
    a = O.Oracle(rig).stitch(frames)
    b = O.Oracle(rig).stitch(frames)
    np.testing.assert_array_equal(a, b)


def strong_perspective_rig(p1=-0.004):
    """three 200 x 120 cameras 160 px apart; camera 2 has a perspective term
    so strong that the top-left 2 x 2 block of its camera-to-canvas matrix has
    a negative determinant while the matrix itself does not (adj[8] < 0 < det)"""
    W, H, step = 200, 120, 160
    cx, cy = (W - 1) / 2, (H - 1) / 2

    def T(tx, ty):
        return np.array([[1, 0, tx], [0, 1, ty], [0, 0, 1.0]])

    Hs = []
    for k in range(3):
        P = np.eye(3)
        if k == 2:
            P[2, 0] = p1
        Hk = T(k * step, 0) @ T(cx, cy) @ P @ T(-cx, -cy)
        Hs.append(Hk / Hk[2, 2])
    H_pair = [np.eye(3)] + [np.linalg.inv(Hs[k - 1]) @ Hs[k] for k in (1, 2)]
    return Hs, dict(n_cams=3, W=W, H=H, ring=0, ring_period=0, canvas_w=560, canvas_h=H, H_pair=H_pair,
                    H_ref=Hs[0])


def test_inverse_keeps_the_front_of_the_camera_when_adj8_is_negative():
    """The canvas-to-camera inverse is a positive multiple of H^-1 (last entry
    +-1), so every pixel of a camera maps back to itself with w > 0 even where
    adj[8] and det differ in sign; dividing by adj[8] alone would flip w."""
    Hs, rig = strong_perspective_rig()
    a = Hs[2]
    assert a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0] < 0 < np.linalg.det(a)
    o = O.Oracle(rig)
    assert o.n_pairs == 2 and o.strip_box(1)[2] > 0
    hinv = np.array(o.plan.hinv[2]).reshape(3, 3)
    assert abs(hinv[2, 2]) == 1.0
    for u in range(2, 198, 13):
        for v in range(2, 118, 11):
            q = a @ np.array([u, v, 1.0])
            ok, uu, vv = O.hom_valid(hinv, q[0] / q[2], q[1] / q[2], 200, 120)
            assert ok and abs(uu - u) < 0.05 and abs(vv - v) < 0.05, (u, v, uu, vv)
