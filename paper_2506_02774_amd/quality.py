"""Image quality metrics for comparing two renders (host side, numpy/scipy).

PSNR, and SSIM as defined by Wang, Bovik, Sheikh and Simoncelli (2004): local
means, variances and covariance under an 11x11 Gaussian window of standard
deviation 1.5, constants C1 = (0.01 L)^2 and C2 = (0.03 L)^2 with dynamic
range L = 1, the SSIM map averaged over the positions where the window lies
inside the image and over the colour channels. Used to report how far the LUT
exponential (Section 4.2) moves the image from the exact one.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import correlate1d

K1, K2, WIN, SIGMA = 0.01, 0.03, 11, 1.5


def gaussian_window(size=WIN, sigma=SIGMA):
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def _local_mean(x, g):
    """Windowed mean at every position where the window fits ('valid')."""
    r = len(g) // 2
    y = correlate1d(correlate1d(x, g, axis=0, mode="constant"), g, axis=1, mode="constant")
    return y[r:x.shape[0] - r, r:x.shape[1] - r]


def ssim_map(a, b, L=1.0):
    """SSIM map of two single-channel images (H, W), H, W >= 11."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    g = gaussian_window()
    c1, c2 = (K1 * L) ** 2, (K2 * L) ** 2
    ma, mb = _local_mean(a, g), _local_mean(b, g)
    saa = _local_mean(a * a, g) - ma * ma
    sbb = _local_mean(b * b, g) - mb * mb
    sab = _local_mean(a * b, g) - ma * mb
    return ((2 * ma * mb + c1) * (2 * sab + c2)) / ((ma * ma + mb * mb + c1) * (saa + sbb + c2))


def ssim(a, b, L=1.0):
    """Mean SSIM of two images (C, H, W) or (H, W)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.ndim == 2:
        return float(ssim_map(a, b, L).mean())
    return float(np.mean([ssim_map(a[c], b[c], L).mean() for c in range(a.shape[0])]))


def psnr(a, b, peak=1.0):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(peak * peak / mse)
