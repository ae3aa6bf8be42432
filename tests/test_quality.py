"""Pins for the image quality metrics (CPU): SSIM against a direct windowed
computation, its closed form on constant images, identity and symmetry; PSNR
of a uniform offset."""
import math

import numpy as np

from paper_2506_02774_amd import quality


def _ssim_direct(a, b):
    """Every window position by explicit weighted sums (the definition)."""
    g = quality.gaussian_window()
    w = np.outer(g, g)
    c1, c2 = (0.01) ** 2, (0.03) ** 2
    H, W = a.shape
    vals = []
    for y in range(H - 10):
        for x in range(W - 10):
            pa, pb = a[y:y + 11, x:x + 11], b[y:y + 11, x:x + 11]
            ma, mb = (w * pa).sum(), (w * pb).sum()
            va, vb = (w * (pa - ma) ** 2).sum(), (w * (pb - mb) ** 2).sum()
            cab = (w * (pa - ma) * (pb - mb)).sum()
            vals.append(((2 * ma * mb + c1) * (2 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    return float(np.mean(vals))


def test_window_is_normalised_gaussian():
    g = quality.gaussian_window()
    assert len(g) == 11 and abs(g.sum() - 1) < 1e-15 and g.argmax() == 5
    np.testing.assert_allclose(g[6] / g[5], math.exp(-1 / (2 * 1.5 ** 2)), rtol=1e-12)


def test_ssim_equals_direct_definition():
    rng = np.random.default_rng(0)
    a = rng.random((19, 23))
    b = np.clip(a + 0.1 * rng.standard_normal(a.shape), 0, 1)
    assert abs(quality.ssim(a, b) - _ssim_direct(a, b)) < 1e-12


def test_ssim_identity_symmetry_and_constants():
    rng = np.random.default_rng(1)
    a = rng.random((3, 24, 30))
    b = rng.random((3, 24, 30))
    assert abs(quality.ssim(a, a) - 1.0) < 1e-12
    assert abs(quality.ssim(a, b) - quality.ssim(b, a)) < 1e-12
    assert quality.ssim(a, b) < 0.5
    # constant images: variances vanish, SSIM = (2 mu_a mu_b + C1) / (mu_a^2 + mu_b^2 + C1)
    ca, cb = np.full((16, 16), 0.3), np.full((16, 16), 0.7)
    c1 = 0.01 ** 2
    assert abs(quality.ssim(ca, cb) - (2 * 0.3 * 0.7 + c1) / (0.09 + 0.49 + c1)) < 1e-12


def test_psnr_uniform_offset():
    a = np.zeros((3, 8, 8))
    assert math.isinf(quality.psnr(a, a))
    assert abs(quality.psnr(a, a + 0.01) - 40.0) < 1e-9
