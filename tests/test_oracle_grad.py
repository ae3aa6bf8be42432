"""Pins for oracle.grad (CPU only): its gradients of sum(w * image) against
central finite differences of oracle.render's numpy image (an independent
code path) on small scenes, element by element, including Gaussians under the
Jacobian clamp, a non-black background and opaque stacks that stop early;
and closed forms for one Gaussian (opacity logit and SH coefficients)."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import scenegen
from oracle import grad, project, render, sh

PARAMS = grad.PARAMS


def _f64(sc, ids=None):
    ids = np.arange(len(sc.mean)) if ids is None else ids
    return SimpleNamespace(mean=sc.mean[ids].astype(np.float64), log_scale=sc.log_scale[ids].astype(np.float64),
                           quat=sc.quat[ids].astype(np.float64), opacity_logit=sc.opacity_logit[ids].astype(np.float64),
                           sh=sc.sh[ids].astype(np.float64).reshape(-1, 16, 3))


def _image(sc, cam, bg, signature=False):
    p = project.project(sc, np.arange(len(sc.mean)), cam)
    return render.render_image(p, cam.width, cam.height, bg=bg, signature=signature)


def _fd_check(sc, cam, bg, gauss, rng, h=1e-6):
    W, H = cam.width, cam.height
    w = rng.normal(size=(3, H, W))
    img, g = grad.image_and_grads(sc, np.arange(len(sc.mean)), cam, w, bg=bg)
    base = _image(sc, cam, bg, signature=True)
    np.testing.assert_allclose(img, base["image"], rtol=0, atol=1e-12)
    checked = 0
    worst = 0.0
    for i in gauss:
        for k in PARAMS:
            arr = getattr(sc, k)
            flat = arr.reshape(len(sc.mean), -1)
            for e in range(flat.shape[1]):
                old = flat[i, e]
                vals = []
                sigs = []
                for s in (1, -1):
                    flat[i, e] = old + s * h
                    r = _image(sc, cam, bg, signature=True)
                    vals.append(float((w * r["image"]).sum()))
                    sigs.append(r["signature"])
                flat[i, e] = old
                if not (np.array_equal(sigs[0], base["signature"]) and np.array_equal(sigs[1], base["signature"])):
                    continue      # the step crossed a blend decision: not differentiable there
                fd = (vals[0] - vals[1]) / (2 * h)
                ad = g[k].reshape(len(sc.mean), -1)[i, e]
                err = abs(fd - ad) / max(1.0, abs(fd))
                worst = max(worst, err)
                assert err <= 1e-6, (k, i, e, fd, ad)
                checked += 1
    return checked, worst


def test_gradients_match_central_differences():
    rng = np.random.default_rng(8)
    sc = _f64(scenegen.random_gaussians(40, 12, 24, 20, depth_range=(2, 8), scale_range=(-2.5, -1.0)))
    cam = scenegen.identity_camera(24, 20)
    n, worst = _fd_check(sc, cam, (0.2, 0.1, 0.3), range(0, 40, 5), rng)
    assert n > 400, n


def test_gradients_under_the_jacobian_clamp():
    """Off-axis Gaussians past 1.3x the half-extent, large enough to reach the
    image: the clamped Jacobian's derivative (the ratio u is constant there)."""
    rng = np.random.default_rng(9)
    n = 12
    z = rng.uniform(3.0, 6.0, n)
    u = rng.choice([-1.0, 1.0], n) * rng.uniform(0.9, 1.3, n)
    mean = np.stack([u * z, rng.uniform(-0.3, 0.3, n) * z, z], 1)
    q = rng.normal(size=(n, 4))
    sc = SimpleNamespace(mean=mean, log_scale=rng.uniform(-0.3, 0.3, (n, 3)), quat=q,
                         opacity_logit=rng.normal(0, 1.5, n), sh=rng.normal(0, 0.2, (n, 16, 3)) + 0.0)
    sc.sh[:, 0] += 0.5
    cam = scenegen.identity_camera(24, 20)
    p = project.project(sc, np.arange(n), cam)
    assert np.all(np.abs(p["mean2d"][:, 0] - 12) / float(np.float32(cam.fx)) > 1.3 * 12 / float(np.float32(cam.fx)))
    cnt, worst = _fd_check(sc, cam, (0.0, 0.0, 0.0), range(n), rng)
    assert cnt > 300, cnt


def test_gradients_with_early_stops():
    """A stack of opaque Gaussians in front of others: pixels stop blending
    (T would fall below 1e-4) and the Gaussians behind get no gradient there."""
    rng = np.random.default_rng(10)
    n = 16
    z = np.linspace(2.0, 4.0, n)
    mean = np.stack([rng.uniform(-0.15, 0.15, n) * z, rng.uniform(-0.15, 0.15, n) * z, z], 1)
    sc = SimpleNamespace(mean=mean, log_scale=np.full((n, 3), -0.5) + rng.uniform(-0.2, 0.2, (n, 3)),
                         quat=rng.normal(size=(n, 4)), opacity_logit=np.full(n, 4.0) + rng.normal(0, 0.3, n),
                         sh=rng.normal(0, 0.2, (n, 16, 3)))
    sc.sh[:, 0] += 0.5
    cam = scenegen.identity_camera(16, 16)
    p = project.project(sc, np.arange(n), cam)
    out = render.render_image(p, 16, 16)
    assert (out["T"] < 1e-3).mean() > 0.2          # many pixels stop
    cnt, worst = _fd_check(sc, cam, (0.5, 0.5, 0.5), range(0, n, 3), rng)
    assert cnt > 200, cnt


def test_single_gaussian_closed_forms():
    """One Gaussian, one pixel (w one-hot): C = alpha c + (1 - alpha) bg with
    alpha = theta e^rho, so dC/dlogit = (1 - theta) alpha (c - bg) and
    dC/dsh_k = alpha Y_k(d) per channel (colour away from its clamp)."""
    cam = scenegen.identity_camera(16, 16)
    sc = SimpleNamespace(mean=np.array([[0.3, -0.2, 4.0]]), log_scale=np.log(np.array([[0.4, 0.3, 0.5]])),
                         quat=np.array([[0.9, 0.1, -0.2, 0.3]]), opacity_logit=np.array([0.4]),
                         sh=np.zeros((1, 16, 3)))
    sc.sh[0, 0] = [0.3, 0.5, 0.7]
    sc.sh[0, 5] = [0.1, -0.1, 0.05]
    bg = np.array([0.1, 0.2, 0.3])
    p = project.project(sc, [0], cam)
    theta = p["theta"][0]
    c = p["rgb"][0]
    Y = sh.basis(sc.mean[0] / np.linalg.norm(sc.mean[0]))
    for (x, y) in [(8, 8), (9, 7), (10, 6)]:
        img = render.render_image(p, 16, 16, bg=bg)["image"]
        alpha = (img[0, y, x] - bg[0]) / (c[0] - bg[0])
        assert 1 / 255 < alpha < 0.99
        for ch in range(3):
            w = np.zeros((3, 16, 16))
            w[ch, y, x] = 1.0
            _, g = grad.image_and_grads(sc, [0], cam, w, bg=bg)
            assert abs(g["opacity_logit"][0] - (1 - theta) * alpha * (c[ch] - bg[ch])) < 1e-12
            want = np.zeros(48)
            want[ch::3] = alpha * Y
            np.testing.assert_allclose(g["sh"][0], want, rtol=1e-12, atol=1e-15)
