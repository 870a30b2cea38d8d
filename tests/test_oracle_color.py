"""Pins of the oracle's colour transfer (section 2.1): histogram
specification (step 3), the least-squares colour matrix of eq. (1), the
3D-M temporal stacking of eqs. (2)-(3) and the state that carries it."""
import numpy as np

from oracle import oracle as O
from paper_2308_09209_amd.scenes import small_scene
from tests.rigs import crop_rig, smooth_image


def hist(v):
    return np.bincount(v.ravel(), minlength=256).astype(np.uint32)


def test_histspec_onto_increasing_map_recovers_the_map():
    rng = np.random.default_rng(0)
    vi = rng.integers(20, 200, 5000)
    g = np.clip(np.round(np.arange(256) * 1.1 + 7), 0, 255).astype(np.int64)  # strictly increasing on [0,200]
    vj = g[vi]
    lut = O.histspec_lut(hist(vi), hist(vj))
    occ = np.unique(vi)
    np.testing.assert_array_equal(lut[occ], g[occ])


def test_histspec_identical_histograms_is_identity_on_occupied_levels():
    rng = np.random.default_rng(1)
    v = rng.integers(0, 256, 3000)
    lut = O.histspec_lut(hist(v), hist(v))
    occ = np.unique(v)
    np.testing.assert_array_equal(lut[occ], occ)


def test_histspec_matches_target_distribution_within_one_level_mass():
    """After specification the cumulative histogram of LUT(i) tracks that of
    j: at every level the gap is at most the largest single-level count."""
    rng = np.random.default_rng(2)
    vi = np.clip(rng.normal(90, 30, 20000), 0, 255).astype(np.int64)
    vj = np.clip(rng.normal(150, 20, 20000), 0, 255).astype(np.int64)
    lut = O.histspec_lut(hist(vi), hist(vj))
    assert np.all(np.diff(lut.astype(int)) >= 0)
    Cs = np.cumsum(hist(lut[vi]).astype(np.int64))
    Cj = np.cumsum(hist(vj).astype(np.int64))
    assert np.max(np.abs(Cs - Cj)) <= max(hist(vi).max(), hist(vj).max())


def test_solve_planted_matrix_exact_normal_equations():
    """Eq. (1) with I_j = I_i M_p: the fit returns M_p (no ridge)."""
    rng = np.random.default_rng(3)
    Ii = rng.integers(10, 200, (4000, 3)).astype(np.float64)   # no clipping of I_i M_p
    Mp = np.eye(3) + rng.uniform(-0.1, 0.1, (3, 3))
    Ij = Ii @ Mp
    M, flag = O.solve_color(Ii.T @ Ii, Ii.T @ Ij, ridge=0.0)
    assert flag == 0
    assert np.max(np.abs(M - Mp)) / np.max(np.abs(Mp)) < 1e-9
    # with the default ridge the pull toward I stays tiny
    M2, _ = O.solve_color(Ii.T @ Ii, Ii.T @ Ij, ridge=1e-9)
    assert np.max(np.abs(M2 - Mp)) < 1e-6
    # byte-rounded target: still recovered to about 1e-2
    M3, _ = O.solve_color(Ii.T @ Ii, Ii.T @ np.floor(Ij + 0.5))
    assert np.max(np.abs(M3 - Mp)) < 1e-2


def test_solve_matches_library_solver():
    rng = np.random.default_rng(4)
    for _ in range(20):
        X = rng.normal(size=(50, 3))
        A = X.T @ X
        B = rng.normal(size=(3, 3)) * 100
        M, flag = O.solve_color(A, B, ridge=0.0)
        assert flag == 0
        np.testing.assert_allclose(M, np.linalg.solve(A, B), rtol=1e-10, atol=1e-10)


def test_solve_equal_moments_is_identity_and_singular_falls_back():
    rng = np.random.default_rng(5)
    Ii = rng.integers(0, 256, (500, 3)).astype(np.float64)
    A = Ii.T @ Ii
    M, flag = O.solve_color(A, A)
    assert flag == 0 and np.max(np.abs(M - np.eye(3))) < 1e-12
    M, flag = O.solve_color(np.zeros((3, 3)), np.zeros((3, 3)))
    assert flag == 1 and np.array_equal(M, np.eye(3))


def test_moments_are_the_normal_equation_products():
    """Tap moments equal I_i^T I_i and I_i^T LUT(I_i) over the mask pixels,
    recomputed in numpy from the strip and LUT taps."""
    s = small_scene(W=120, H=72)
    o = O.Oracle(s.rig())
    o.stitch(s.frames(0))
    for p in range(o.n_pairs):
        m = o.tap("mask", p).astype(bool)
        Ii = o.tap("strip", p, 1)[m].astype(np.uint64)
        lut = o.tap("lut", p)
        Q = np.stack([lut[c][Ii[:, c]] for c in range(3)], 1).astype(np.uint64)
        A = Ii.T @ Ii
        B = Ii.T @ Q
        mom = o.tap("mom", p)
        np.testing.assert_array_equal(mom[:6], A[np.triu_indices(3)])
        np.testing.assert_array_equal(mom[6:15], B.ravel())
        assert mom[15] == m.sum()
        # the histograms are those of the masked strips
        h = o.tap("hist", p)
        Ij = o.tap("strip", p, 0)[m]
        for c in range(3):
            np.testing.assert_array_equal(h[1, c], np.bincount(Ii[:, c].astype(int), minlength=256))
            np.testing.assert_array_equal(h[0, c], np.bincount(Ij[:, c], minlength=256))


def _solve_from(moms, ridge=1e-9):
    A = np.zeros(6)
    B = np.zeros(9)
    for m in moms:
        A += m[:6].astype(np.float64)
        B += m[6:15].astype(np.float64)
    As = np.array([[A[0], A[1], A[2]], [A[1], A[3], A[4]], [A[2], A[4], A[5]]])
    return O.solve_color(As, B.reshape(3, 3), ridge)[0]


def test_3dm_window_uses_frames_T_T1_T2():
    """Eqs. (2)-(3): the matrix of frame T solves the summed moments of
    frames T, T-1, T-2 (frames before 0 absent, eq. (6)-(7) analogue)."""
    s = small_scene(W=120, H=72, drift=0.05)
    o = O.Oracle(s.rig())
    moms, mp = [], []
    for t in range(5):
        o.stitch(s.frames(t))
        moms.append(o.tap("mom", 0))
        mp.append(o.tap("mpair")[0])
    for t in range(5):
        ref = _solve_from(moms[max(0, t - 2):t + 1])
        np.testing.assert_allclose(mp[t], ref, rtol=0, atol=1e-12)


def test_3dm_with_repeated_frames_equals_2dm():
    s = small_scene(W=120, H=72)
    f = s.frames(0)
    o3 = O.Oracle(s.rig(), color_window=3)
    o1 = O.Oracle(s.rig(), color_window=1)
    for _ in range(3):
        o3.stitch(f)
        o1.stitch(f)
    np.testing.assert_allclose(o3.tap("mpair"), o1.tap("mpair"), rtol=1e-12, atol=1e-14)


def test_chain_composition_maps_every_camera_to_camera_0():
    s = small_scene(n_cams=3, W=100, H=64)
    o = O.Oracle(s.rig())
    o.stitch(s.frames(0))
    mp = o.tap("mpair")
    mk = o.tap("mk")
    np.testing.assert_array_equal(mk[0], np.eye(3, dtype=np.float32))
    np.testing.assert_allclose(mk[1], mp[0], rtol=1e-6)
    np.testing.assert_allclose(mk[2], mp[1] @ mp[0], rtol=1e-6, atol=1e-7)


def test_planted_gain_recovered_end_to_end():
    """Camera 1 sees the same texture through a planted per-channel gain:
    the fitted pair matrix is that gain (to byte rounding)."""
    tex = smooth_image(64, 220, seed=21)
    rig, frames = crop_rig(tex, 120, 64, [(0, 0), (100, 0)])
    gain = np.array([0.8, 1.0, 1.15])
    # camera j = 0 sees tex * gain; camera i = 1 sees tex: M maps i -> j
    frames[0] = np.clip(np.floor(frames[0] * gain + 0.5), 0, 255).astype(np.uint8)
    o = O.Oracle(rig, balance=0)
    o.stitch(frames)
    M = o.tap("mpair")[0]
    np.testing.assert_allclose(M, np.diag(gain), atol=2e-2)
