"""Pins for oracle.sh (CPU only): scipy's complex spherical harmonics converted
to the real basis, orthonormality under quadrature, and the degree-0 colour."""
import math

import numpy as np
import scipy.special as sps

from oracle import sh


def _real_from_scipy(l, m, polar, azim):
    if hasattr(sps, "sph_harm_y"):
        Y = sps.sph_harm_y(l, abs(m), polar, azim)
    else:  # older scipy: sph_harm(m, n, azimuth, polar)
        Y = sps.sph_harm(abs(m), l, azim, polar)
    if m == 0:
        return Y.real
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * Y.real
    return math.sqrt(2.0) * (-1) ** m * Y.imag


def test_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    polar = np.arccos(np.clip(d[:, 2], -1, 1))
    azim = np.arctan2(d[:, 1], d[:, 0])
    B = sh.basis(d)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _real_from_scipy(l, m, polar, azim)
            np.testing.assert_allclose(B[:, l * l + l + m], ref, atol=1e-12, err_msg=f"l={l} m={m}")


def test_orthonormal_quadrature():
    # Gauss-Legendre in cos(polar) x uniform azimuth integrates degree <= 6 polynomials exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    na = 24
    az = (np.arange(na) + 0.5) * 2 * math.pi / na
    ct, A = np.meshgrid(xg, az, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(A), st * np.sin(A), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(na, 2 * math.pi / na)[None, :]).ravel()
    B = sh.basis(d)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_degree0_colour_and_clamp():
    c = np.zeros((2, 16, 3))
    c[0, 0] = [0.5, -0.2, 10.0]
    c[1, 0] = [0.0, 0.0, 0.0]
    rgb = sh.colour(c, np.array([[0.0, 0.0, 3.0], [1.0, 2.0, 3.0]]))
    y0 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(rgb[0], [y0 * 0.5 + 0.5, y0 * -0.2 + 0.5, 1.0], atol=1e-15)
    np.testing.assert_allclose(rgb[1], [0.5, 0.5, 0.5], atol=1e-15)
