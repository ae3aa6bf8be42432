"""Pins for oracle.render (CPU only): one- and two-Gaussian closed forms, an
opaque stack's termination count, depth ties ordered by id, and the
vectorised blend against the literal per-pixel loop on small random scenes."""
import math

import numpy as np

import scenegen
from oracle import project, render


def _proj(mx, my, conic, theta, rgb, depth, ids=None):
    n = len(mx)
    return dict(ids=np.arange(n) if ids is None else np.asarray(ids), valid=np.ones(n, bool),
                mean2d=np.stack([mx, my], 1).astype(float), conic=np.asarray(conic, float),
                theta=np.asarray(theta, float), rgb=np.asarray(rgb, float), depth=np.asarray(depth, float),
                radius=np.full(n, 1e6), near_margin=np.ones(n))


def test_single_gaussian_closed_form():
    p = _proj([8.0], [8.0], [[0.02, 0.005, 0.03]], [0.7], [[0.2, 0.4, 0.9]], [3.0])
    out = render.render_image(p, 16, 16, bg=(0.1, 0.0, 0.3))
    for (x, y) in [(8, 8), (2, 5), (15, 0), (7, 12)]:
        dx, dy = x + 0.5 - 8.0, y + 0.5 - 8.0
        a = min(0.99, 0.7 * math.exp(-0.5 * (0.02 * dx * dx + 0.01 * dx * dy + 0.03 * dy * dy)))
        exp = (np.array([0.2, 0.4, 0.9]) * a + (1 - a) * np.array([0.1, 0, 0.3])) if a >= 1 / 255 \
            else np.array([0.1, 0, 0.3])
        np.testing.assert_allclose(out["image"][:, y, x], exp, atol=1e-14)


def test_two_gaussians_depth_order():
    # the nearer one (depth 2) is blended first regardless of list order
    p = _proj([4.0, 4.0], [4.0, 4.0], [[1e-6, 0, 1e-6]] * 2, [0.6, 0.5], [[1, 0, 0], [0, 1, 0]], [5.0, 2.0])
    c = render.render_pixels(p, [3], [3])["rgb"][0]
    a1, a2 = 0.5, 0.6     # rho ~ 0 at the centre
    np.testing.assert_allclose(c, [a2 * (1 - a1), a1, 0.0], atol=1e-5)


def test_opaque_stack_termination():
    # eight alpha = 0.8 Gaussians: T = 0.2^k; the 6th would take T to 6.4e-5 < 1e-4 -> 5 blended
    n = 8
    p = _proj([0.5] * n, [0.5] * n, [[1e-9, 0, 1e-9]] * n, [0.8] * n, [[1, 1, 1]] * n, np.arange(1, n + 1))
    r = render.render_pixels(p, [0], [0])
    assert r["n_contrib"][0] == 5
    np.testing.assert_allclose(r["rgb"][0], [1 - 0.2 ** 5] * 3, atol=1e-9)
    np.testing.assert_allclose(r["T"][0], 0.2 ** 5, rtol=1e-6)
    # Eq. 3's 0.99 clamp: theta = 1 at the centre still gives alpha = 0.99
    p = _proj([0.5], [0.5], [[1e-9, 0, 1e-9]], [1.0], [[1, 0, 0]], [1.0])
    r = render.render_pixels(p, [0], [0])
    np.testing.assert_allclose(r["rgb"][0], [0.99, 0, 0], atol=1e-9)


def test_ambiguity_flags():
    # alpha exactly at alpha* (within 1e-6) at the centre pixel is flagged, a clear one is not
    p = _proj([0.5, 5.5], [0.5, 0.5], [[1e-12, 0, 1e-12]] * 2, [1 / 255 * (1 + 1e-6), 0.5], [[1, 1, 1]] * 2,
              [1.0, 2.0])
    p["radius"][:] = 1.0
    r = render.render_pixels(p, [0, 5], [0, 0])
    assert r["ambiguous"].tolist() == [True, False]


def test_equal_depth_ordered_by_id():
    p = _proj([2.0, 2.0], [2.0, 2.0], [[1e-6, 0, 1e-6]] * 2, [0.5, 0.5], [[1, 0, 0], [0, 1, 0]], [4.0, 4.0],
              ids=[9, 3])
    c = render.render_pixels(p, [1], [1])["rgb"][0]
    # id 3 (green) first
    np.testing.assert_allclose(c, [0.25, 0.5, 0.0], atol=1e-5)


def test_vectorised_equals_loop():
    sc = scenegen.random_gaussians(60, 1, 32, 24, depth_range=(2, 10), scale_range=(-3.0, -1.0))
    cam = scenegen.identity_camera(32, 24)
    p = project.project(sc, np.arange(60), cam)
    out = render.render_image(p, 32, 24, bg=(0.2, 0.3, 0.4), chunk=7)
    rng = np.random.default_rng(0)
    for _ in range(40):
        x, y = int(rng.integers(32)), int(rng.integers(24))
        c, T, n = render.render_pixel_loop(p, x, y, bg=(0.2, 0.3, 0.4))
        np.testing.assert_allclose(out["image"][:, y, x], c, atol=1e-12)
        assert out["n_contrib"][y, x] == n
        np.testing.assert_allclose(out["T"][y, x], T, rtol=1e-12)
