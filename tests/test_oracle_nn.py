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
