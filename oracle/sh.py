"""Oracle: real spherical harmonics up to degree 3 (FP64). Test infrastructure only.

The paper renders 3DGS Gaussians, whose view-dependent colour is a degree-3
spherical-harmonic expansion; it does not state the convention. Reading used:
real, orthonormal SH on the unit sphere without the Condon-Shortley phase,
coefficient index k = l*l + l + m (m = -l..l), colour = sum_k c_k Y_k(d) + 0.5,
clamped to [0, 1], with d the unit vector from the camera centre to the mean.

Pinned by tests/test_oracle_sh.py against scipy's complex spherical harmonics
(real part / imaginary part conversion) and by orthonormality under quadrature.
"""
from __future__ import annotations

import math

import numpy as np

_PI = math.pi
# normalisation constants written from K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), times sqrt(2) for m != 0
C0 = 0.5 * math.sqrt(1.0 / _PI)
C1 = math.sqrt(3.0 / (4.0 * _PI))
C2_xy = 0.5 * math.sqrt(15.0 / _PI)
C2_0 = 0.25 * math.sqrt(5.0 / _PI)
C2_2 = 0.25 * math.sqrt(15.0 / _PI)
C3_3 = 0.25 * math.sqrt(35.0 / (2.0 * _PI))
C3_2m = 0.5 * math.sqrt(105.0 / _PI)
C3_1 = 0.25 * math.sqrt(21.0 / (2.0 * _PI))
C3_0 = 0.25 * math.sqrt(7.0 / _PI)
C3_2p = 0.25 * math.sqrt(105.0 / _PI)


def basis(d: np.ndarray) -> np.ndarray:
    """Y_k(d) for unit vectors d (..., 3) -> (..., 16)."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    xx, yy, zz = x * x, y * y, z * z
    r2 = xx + yy + zz
    out = np.empty(d.shape[:-1] + (16,), np.float64)
    out[..., 0] = C0
    out[..., 1] = C1 * y
    out[..., 2] = C1 * z
    out[..., 3] = C1 * x
    out[..., 4] = C2_xy * x * y
    out[..., 5] = C2_xy * y * z
    out[..., 6] = C2_0 * (3.0 * zz - r2)
    out[..., 7] = C2_xy * x * z
    out[..., 8] = C2_2 * (xx - yy)
    out[..., 9] = C3_3 * y * (3.0 * xx - yy)
    out[..., 10] = C3_2m * x * y * z
    out[..., 11] = C3_1 * y * (5.0 * zz - r2)
    out[..., 12] = C3_0 * z * (5.0 * zz - 3.0 * r2)
    out[..., 13] = C3_1 * x * (5.0 * zz - r2)
    out[..., 14] = C3_2p * z * (xx - yy)
    out[..., 15] = C3_3 * x * (xx - 3.0 * yy)
    return out


def colour(coeffs: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """RGB in [0, 1] from SH coefficients (n, 16, 3) and view directions (n, 3)
    (camera centre -> Gaussian mean, any length)."""
    d = np.asarray(dirs, np.float64)
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    Y = basis(d)
    rgb = np.einsum("nk,nkc->nc", Y, np.asarray(coeffs, np.float64)) + 0.5
    return np.clip(rgb, 0.0, 1.0)
