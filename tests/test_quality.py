"""Host checks of the quality harness (paper_2308_09209_amd/quality.py): its
PSNR and SSIM against closed forms and a direct window sum, and the
generator's ground-truth panorama against the camera frames of a rig whose
cameras are exact crops with no colour response."""
import numpy as np

from paper_2308_09209_amd import quality as Q
from paper_2308_09209_amd.scenes import Scene


def test_psnr_closed_form():
    a = np.full((10, 12, 3), 100, np.uint8)
    for d in (1, 5, 17):
        b = a + np.uint8(d)
        assert abs(Q.psnr(a, b) - 10 * np.log10(255.0 ** 2 / d ** 2)) < 1e-12
    m = np.zeros((10, 12), bool)
    m[2:5, 3:9] = True
    b = a.copy()
    b[~m] = 0
    assert Q.psnr(a, b, m) == float("inf")


def test_ssim_identical_and_constant_images():
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 255, (40, 50))
    assert np.allclose(Q.ssim_map(a, a), 1.0)
    # constant images: no variance, SSIM = (2 a b + C1) / (a^2 + b^2 + C1)
    C1 = (0.01 * 255) ** 2
    m = Q.ssim_map(np.full((20, 20), 80.0), np.full((20, 20), 120.0))
    assert np.allclose(m, (2 * 80 * 120 + C1) / (80 ** 2 + 120 ** 2 + C1))


def test_ssim_matches_a_direct_window_sum():
    rng = np.random.default_rng(2)
    a = rng.uniform(0, 255, (30, 30))
    b = np.clip(a + rng.normal(0, 20, a.shape), 0, 255)
    r = np.arange(-5, 6)
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2 * 1.5 ** 2))
    g /= g.sum()
    y, x = 14, 17
    wa, wb = a[y - 5:y + 6, x - 5:x + 6], b[y - 5:y + 6, x - 5:x + 6]
    ma, mb = (g * wa).sum(), (g * wb).sum()
    va = (g * wa * wa).sum() - ma * ma
    vb = (g * wb * wb).sum() - mb * mb
    cab = (g * wa * wb).sum() - ma * mb
    C1, C2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    want = (2 * ma * mb + C1) * (2 * cab + C2) / ((ma * ma + mb * mb + C1) * (va + vb + C2))
    assert abs(Q.ssim_map(a, b)[y, x] - want) < 1e-10


def test_truth_panorama_equals_exact_crops():
    sc = Scene(n_cams=3, W=64, H=48, overlap=0.3, ring=False, tex_h=100, resid=0.0, perturb=False, colour=False)
    truth = sc.truth(0)
    for k, f in enumerate(sc.frames(0)):
        np.testing.assert_array_equal(truth[:, k * sc.step:k * sc.step + sc.W], f)
