"""Pins of the FP64 convolution references used to check the surrogate's
matrix-core kernels (a library correlation and finite differences)."""
import numpy as np
from scipy.signal import correlate2d

from oracle import oracle as O


def test_conv3x3_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 7, 9, 3))
    wt = rng.normal(size=(4, 9, 3))
    b = rng.normal(size=4)
    y = O.conv3x3(x, wt, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(correlate2d(x[n, :, :, ci], wt[co, :, ci].reshape(3, 3), mode="same")
                              for ci in range(3))
            np.testing.assert_allclose(y[n, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_conv3x3_gradients_by_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 5, 6, 2))
    wt = rng.normal(size=(3, 9, 2))
    b = rng.normal(size=3)
    r = rng.normal(size=(1, 5, 6, 3))          # L = sum(conv(x) * r)
    dx = O.conv3x3_bwd_data(r, wt)
    dw, db = O.conv3x3_bwd_weight(x, r)
    L = lambda xx, ww, bb: float((O.conv3x3(xx, ww, bb) * r).sum())
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (0, 2, 3, 1), (0, 4, 5, 0), (0, 1, 5, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert abs((L(xp, wt, b) - L(xm, wt, b)) / (2 * eps) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0), (2, 4, 1), (1, 8, 0), (0, 6, 1)]:
        wp, wm = wt.copy(), wt.copy()
        wp[idx] += eps
        wm[idx] -= eps
        assert abs((L(x, wp, b) - L(x, wm, b)) / (2 * eps) - dw[idx]) < 1e-6
    for co in range(3):
        bp, bm = b.copy(), b.copy()
        bp[co] += eps
        bm[co] -= eps
        assert abs((L(x, wt, bp) - L(x, wt, bm)) / (2 * eps) - db[co]) < 1e-6


def test_network_step_forward_closed_form():
    """Two layers whose only weights are identity centre taps: the output is
    b2 + lrelu(x + b1) channel by channel, so a dropped activation, a wrong
    slope or a swapped layer order changes it."""
    rng = np.random.default_rng(4)
    sizes = [(3, 4), (2, 5)]
    P = sum(h * w for h, w in sizes)
    x = rng.normal(size=(P, 2))
    w1 = np.zeros((2, 9, 2))
    w2 = np.zeros((2, 9, 2))
    for c in range(2):
        w1[c, 4, c] = 1.0
        w2[c, 4, c] = 1.0
    b1, b2 = np.array([0.3, -0.2]), np.array([1.0, 2.0])
    label = rng.normal(size=(P, 2))
    loss, pred, _, _ = O.nn_train_step([w1, w2], [b1, b2], x, label, sizes, 0.1)
    z = x + b1
    want = np.where(z > 0, z, 0.1 * z) + b2
    np.testing.assert_allclose(pred, want, rtol=0, atol=1e-14)
    d = want - label
    assert abs(loss - np.mean(np.sqrt((d ** 2).sum(1) + 1e-6))) < 1e-14


def test_network_step_gradients_by_finite_differences():
    """The whole chain's gradients (loss -> last layer -> leaky ReLU -> first
    layer, over two images) against central differences of the loss."""
    rng = np.random.default_rng(5)
    sizes = [(4, 5), (3, 3)]
    P = sum(h * w for h, w in sizes)
    ws = [rng.normal(size=(3, 9, 2)) * 0.5, rng.normal(size=(3, 9, 3)) * 0.5, rng.normal(size=(2, 9, 3)) * 0.5]
    bs = [rng.normal(size=3) * 0.1, rng.normal(size=3) * 0.1, rng.normal(size=2) * 0.1]
    x = rng.normal(size=(P, 2))
    label = rng.normal(size=(P, 2))
    _, _, gw, gb = O.nn_train_step(ws, bs, x, label, sizes, 0.1)
    eps = 1e-6

    def loss_with(li, kind, idx, delta):
        w2 = [w.copy() for w in ws]
        b2 = [b.copy() for b in bs]
        (w2 if kind == "w" else b2)[li][idx] += delta
        return O.nn_train_step(w2, b2, x, label, sizes, 0.1)[0]

    for li in range(3):
        for idx in [(0, 0, 0), (1, 4, 1), (ws[li].shape[0] - 1, 8, ws[li].shape[2] - 1)]:
            fd = (loss_with(li, "w", idx, eps) - loss_with(li, "w", idx, -eps)) / (2 * eps)
            assert abs(fd - gw[li][idx]) < 1e-7, (li, idx, fd, gw[li][idx])
        for co in range(bs[li].shape[0]):
            fd = (loss_with(li, "b", co, eps) - loss_with(li, "b", co, -eps)) / (2 * eps)
            assert abs(fd - gb[li][co]) < 1e-7, (li, co)
