"""Pins of the oracle's learned-surrogate flow path (CPU).

The surrogate is not in the paper; what fixes it is its own definition: a
chain of zero-padded 3x3 cross-correlations with BF16 storage between layers,
a x4 bilinear upsampling to level 0 and a forward-backward consistency check.
Each pin below is fixed by something other than the oracle itself: an
independent library routine (scipy's 2-D correlation), closed forms on dyadic
values where every rounding is exact, or invariants of the pipeline (a zero
threshold reproduces the plain estimator bit for bit; a zero network
reproduces the zero-flow stitcher)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import oracle as O
from paper_2308_09209_amd import scenes as S


def bf16(x):
    return (S.bf16_bits(x).view(np.uint16).astype(np.uint32) << 16).view(np.float32)


def one_hot_net(layers, entries, alpha=0.1, biases=None):
    """weights zero except entries[(layer, co, tap, ci)] = value"""
    ws = [np.zeros((co, 9, ci)) for (ci, co) in layers]
    for (l, co, tap, ci), v in entries.items():
        ws[l][co, tap, ci] = v
    bs = biases or [np.zeros(co) for (_, co) in layers]
    return S.nn_blob(ws, bs, alpha)


def luma(h, w, seed):
    return np.random.default_rng(seed).integers(0, 256, size=(h, w)).astype(np.float32)


# ---- the network ------------------------------------------------------------

@pytest.mark.parametrize("layers", [((16, 32), (32, 16)), S.SURROGATE_LAYERS])
def test_network_is_a_chain_of_scipy_correlations(layers):
    ws, bs = S.random_net(7, layers)
    blob = S.nn_blob(ws, bs, 0.1)
    yt = luma(11, 17, 1) + np.float32(0.25)
    ym = luma(11, 17, 2) - np.float32(0.5)
    got = O.surrogate_net(blob, yt, ym)
    # independent evaluation: scipy's 'same' 2-D correlation per (cout, cin)
    x = np.zeros((11, 17, layers[0][0]))
    x[:, :, 0] = bf16((yt - np.float32(128)) * np.float32(1 / 64))
    x[:, :, 1] = bf16((ym - np.float32(128)) * np.float32(1 / 64))
    for li, (ci, co) in enumerate(layers):
        wq = bf16(ws[li]).astype(np.float64)
        y = np.zeros((11, 17, co))
        for o in range(co):
            acc = np.full((11, 17), np.float64(np.float32(bs[li][o])))
            for c in range(ci):
                acc += correlate2d(x[:, :, c], wq[o, :, c].reshape(3, 3), mode="same", boundary="fill")
            y[:, :, o] = acc
        y = y.astype(np.float32)
        if li < len(layers) - 1:
            y = np.where(y > 0, y, np.float32(0.1) * y).astype(np.float32)
            x = bf16(y).astype(np.float64)
        else:
            want = y[:, :, :2]
    assert np.abs(got - want).max() <= 1e-6 * (1 + np.abs(want).max())


def test_input_encoding_and_tap_orientation():
    # output channel 0 reads channel 0 (template) through tap 2 = (ky 0, kx 2),
    # i.e. pixel (y - 1, x + 1); channel 1 reads the moving image's centre tap
    blob = one_hot_net(((16, 16),), {(0, 0, 2, 0): 1.0, (0, 1, 4, 1): 1.0})
    yt, ym = luma(6, 9, 3), luma(6, 9, 4)
    got = O.surrogate_net(blob, yt, ym)
    enc_t = (yt - 128.0) / 64.0          # exact: integer luma has <= 8 significant bits
    enc_m = (ym - 128.0) / 64.0
    want0 = np.zeros_like(enc_t)
    want0[1:, :-1] = enc_t[:-1, 1:]
    assert np.array_equal(got[:, :, 0], want0)
    assert np.array_equal(got[:, :, 1], enc_m)


def test_leaky_relu_on_hidden_layers_closed_form():
    # h0 = x, h1 = -x, then out = lrelu(h0) - lrelu(h1) = (1 + alpha) x for any x
    blob = one_hot_net(((16, 16), (16, 16)),
                       {(0, 0, 4, 0): 1.0, (0, 1, 4, 0): -1.0, (1, 0, 4, 0): 1.0, (1, 0, 4, 1): -1.0},
                       alpha=0.5)
    yt = luma(5, 7, 5)
    got = O.surrogate_net(blob, yt, yt)
    assert np.array_equal(got[:, :, 0], 1.5 * (yt - 128.0) / 64.0)
    assert np.all(got[:, :, 1] == 0)


# ---- upsampling and the forward-backward check ------------------------------

def test_upsampling_reproduces_a_linear_field():
    h2, w2, h0, w0 = 6, 8, 24, 30
    Y, X = np.mgrid[0:h2, 0:w2].astype(np.float64)
    pred = np.stack([0.5 * X + 0.25, -0.25 * Y + 1.0], axis=-1).astype(np.float32)
    need = np.ones((h0, w0), np.uint8)
    need[3, 5] = 0
    got = O.surr_upsample(pred, need)
    y0, x0 = np.mgrid[0:h0, 0:w0].astype(np.float64)
    cx = np.clip(x0 / 4 - 0.375, 0, w2 - 1)
    cy = np.clip(y0 / 4 - 0.375, 0, h2 - 1)
    want = np.stack([4 * (0.5 * cx + 0.25), 4 * (-0.25 * cy + 1.0)], axis=-1)
    want[3, 5] = 0.0
    assert np.array_equal(got, want.astype(np.float32))


def test_forward_backward_error_closed_forms():
    h2, w2 = 5, 9
    need = np.zeros((20, 36), np.uint8)
    need[2:18, 3:30] = 1
    n = int(need.sum())
    a = np.tile(np.float32([0.25, -0.5]), (h2, w2, 1))
    # exact inverse: zero error
    assert O.fb_check(a, -a, need) == (0, n)
    # a constant mismatch of 0.125 level-2 px = 0.5 px: 128 / 256 px per pixel
    b = -a.copy()
    b[:, :, 0] += 0.125
    assert O.fb_check(a, b, need) == (128 * n, n)
    # the same field both ways: e = 2 |U|, U = (1, -2) px
    s, cnt = O.fb_check(a, a, need)
    assert cnt == n and s == n * int(np.floor(2 * np.sqrt(5.0) * 256 + 0.5))
    # a non-finite prediction saturates at 2^20 per pixel
    c = a.copy()
    c[:] = np.nan
    assert O.fb_check(c, a, need) == (n << 20, n)


def test_backward_flow_is_read_at_the_displaced_point():
    # U_ij = (4, 0) px everywhere; U_ji(x) = 4 (0.25 (x / 4 - 0.375) - 1) in the
    # interior, so e(x) = |4 + U_ji(x + 4)| = |0.25 x + 0.625| (read at x it
    # would be |0.25 x - 0.375|)
    h2, w2 = 4, 12
    Y, X = np.mgrid[0:h2, 0:w2].astype(np.float64)
    pij = np.zeros((h2, w2, 2), np.float32)
    pij[:, :, 0] = 1.0
    pji = np.zeros((h2, w2, 2), np.float32)
    pji[:, :, 0] = 0.25 * X - 1.0
    need = np.zeros((16, 48), np.uint8)
    need[:, 2:38] = 1                      # x / 4 - 0.375 >= 0 and (x + 4) / 4 - 0.375 <= w2 - 1
    s, n = O.fb_check(pij, pji, need)
    xs = np.arange(2, 38, dtype=np.float64)
    want = 16 * int(np.floor(np.abs(0.25 * xs + 0.625) * 256 + 0.5).sum())
    assert n == 16 * 36 and s == want


# ---- inside the frame ---------------------------------------------------------

def _run(scene, frames, blob=None, mode=0, tau=0.0, **params):
    o = O.Oracle(scene.rig(), **params)
    if blob is not None or mode:
        o.set_surrogate(blob, mode, tau)
    panos = [o.stitch(scene.frames(t)) for t in range(frames)]
    return o, panos


@pytest.fixture(scope="module")
def scene():
    return S.small_scene(n_cams=3, W=96, H=64, overlap=0.35, ring=True, seed_config=91)


def test_zero_threshold_falls_back_to_the_plain_flow_bit_for_bit(scene):
    ws, bs = S.random_net(3)
    o_plain, p_plain = _run(scene, 3)
    o_fb, p_fb = _run(scene, 3, S.nn_blob(ws, bs), O.FLOW_FALLBACK, 0.0)
    for a, b in zip(p_plain, p_fb):
        assert np.array_equal(a, b)
    assert np.all(o_fb.tap("surr_ok") == 0)
    for p in range(o_plain.n_pairs):
        for d in range(2):
            assert np.array_equal(o_plain.tap("flow", p, d), o_fb.tap("flow", p, d))


def test_zero_network_gives_the_zero_flow_stitch(scene):
    layers = S.SURROGATE_LAYERS
    blob = S.nn_blob([np.zeros((co, 9, ci)) for ci, co in layers], [np.zeros(co) for _, co in layers])
    _, p_zero = _run(scene, 2, flow=0)
    o, p_surr = _run(scene, 2, blob, O.FLOW_SURROGATE)
    for a, b in zip(p_zero, p_surr):
        assert np.array_equal(a, b)
    assert np.all(o.tap("surr_ok") == 1)


def test_bias_only_network_and_the_strict_threshold(scene):
    layers = S.SURROGATE_LAYERS
    ws = [np.zeros((co, 9, ci)) for ci, co in layers]
    bs = [np.zeros(co) for _, co in layers]
    bs[-1][0] = 0.25                       # 1 px at level 0, the same both ways
    blob = S.nn_blob(ws, bs)
    o, _ = _run(scene, 1, blob, O.FLOW_SURROGATE)
    for p in range(o.n_pairs):
        need = o.tap("need", p, 0).astype(bool)
        for d in range(2):
            f = o.tap("flow", p, d)
            assert np.all(f[need] == np.float32([1.0, 0.0])) and np.all(f[~need] == 0)
        s, n = o.tap("fb")[p]
        assert n == need.sum() and s == 512 * n          # e = |1 + 1| = 2 px
    o2, _ = _run(scene, 1, blob, O.FLOW_FALLBACK, 2.0)   # mean error 2 px is not below 2 px
    assert np.all(o2.tap("surr_ok") == 0)
    o3, _ = _run(scene, 1, blob, O.FLOW_FALLBACK, 2.01)
    assert np.all(o3.tap("surr_ok") == 1)


def test_large_threshold_equals_surrogate_only(scene):
    ws, bs = S.random_net(5)
    blob = S.nn_blob(ws, bs)
    o1, p1 = _run(scene, 2, blob, O.FLOW_SURROGATE)
    o2, p2 = _run(scene, 2, blob, O.FLOW_FALLBACK, 1e6)
    for a, b in zip(p1, p2):
        assert np.array_equal(a, b)
    assert np.array_equal(o1.tap("fb"), o2.tap("fb"))
    for p in range(o1.n_pairs):
        need = o1.tap("need", p, 0)
        want = O.surr_upsample(o1.tap("surr_pred", p, 0), need)
        assert np.array_equal(o1.tap("flow", p, 0), want)


def test_surrogate_needs_weights_and_three_levels(scene):
    o = O.Oracle(scene.rig())
    with pytest.raises(O.OracleError):
        o.set_surrogate(None, O.FLOW_SURROGATE)
    with pytest.raises(O.OracleError):
        o.set_surrogate(b"VSNN" + b"\0" * 12, O.FLOW_SURROGATE)
    ws, bs = S.random_net(1)
    o2 = O.Oracle(scene.rig(), lk_levels=2)
    with pytest.raises(O.OracleError):
        o2.set_surrogate(S.nn_blob(ws, bs), O.FLOW_SURROGATE)
