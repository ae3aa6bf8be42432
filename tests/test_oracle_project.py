"""Pins for oracle.project (CPU only): closed forms for an isotropic on-axis
Gaussian, the Jacobian against finite differences of the pinhole map,
covariance determinant and quaternion-sign invariance, culling at the near plane."""
import math

import numpy as np

import scenegen
from oracle import project


def _one(mean, log_scale, quat=(1, 0, 0, 0), logit=0.0):
    sc = scenegen.tree_from_arrays([-1], [-1], [0], [[0, 0, 0]], [[0, 0, 0]], mean=[mean], log_scale=[log_scale],
                                   quat=[quat], opacity_logit=[logit])
    return sc


def test_isotropic_on_axis_closed_form():
    cam = scenegen.identity_camera(256, 256)
    f = float(np.float32(cam.fx))
    for z, sig in [(5.0, 0.3), (20.0, 1.0), (2.0, 0.05)]:
        sc = _one([0.0, 0.0, z], [math.log(sig)] * 3)
        p = project.project(sc, [0], cam)
        v = (f * sig / z) ** 2 + 0.3
        np.testing.assert_allclose(p["cov2d"][0], [v, 0.0, v], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(p["conic"][0], [1 / v, 0.0, 1 / v], rtol=1e-6, atol=1e-12)
        np.testing.assert_allclose(p["mean2d"][0], [128.0, 128.0], atol=1e-12)
        assert p["radius"][0] == math.ceil(3.33 * math.sqrt(v))
        assert p["depth"][0] == z and p["valid"][0]


def test_jacobian_vs_finite_differences():
    rng = np.random.default_rng(3)
    cam = scenegen.look_camera([1.0, -2.0, 1.7], 0.4, -0.1, 320, 240)
    R = cam.R.astype(np.float64)
    pos = cam.pos.astype(np.float64)
    f = float(np.float32(cam.fx))

    def pix(x):
        c = R @ (x - pos)
        return np.array([f * c[0] / c[2] + cam.cx, f * c[1] / c[2] + cam.cy])

    for _ in range(20):
        fwd = R[2]
        mu = pos + fwd * rng.uniform(3, 30) + rng.normal(size=3) * 0.5
        ls = rng.uniform(-2.5, 0.0, 3)
        q = rng.normal(size=4)
        sc = _one(mu, ls, q)
        p = project.project(sc, [0], cam)
        mu32 = sc.mean[0].astype(np.float64)
        Jn = np.zeros((2, 3))
        h = 1e-5
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (pix(mu32 + e) - pix(mu32 - e)) / (2 * h)
        S3 = project.covariance3d(sc.log_scale, sc.quat)[0]
        S2 = Jn @ S3 @ Jn.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(p["cov2d"][0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(p["mean2d"][0], pix(mu32), rtol=1e-12)


def test_covariance_properties():
    rng = np.random.default_rng(5)
    ls = rng.uniform(-3, 1, (50, 3))
    q = rng.normal(size=(50, 4))
    S = project.covariance3d(ls, q)
    np.testing.assert_allclose(np.linalg.det(S), np.exp(2 * ls.sum(1)), rtol=1e-9)
    np.testing.assert_allclose(project.covariance3d(ls, -q), S, atol=1e-12)
    # eigenvalues are the squared scales
    ev = np.sort(np.linalg.eigvalsh(S), axis=1)
    np.testing.assert_allclose(ev, np.sort(np.exp(2 * ls), axis=1), rtol=1e-9)


def test_near_plane_and_opacity():
    cam = scenegen.identity_camera(64, 64)
    sc = _one([0.0, 0.0, 0.19], [-2.0] * 3, logit=1.3)
    assert not project.project(sc, [0], cam)["valid"][0]
    sc = _one([0.0, 0.0, 0.21], [-2.0] * 3, logit=1.3)
    p = project.project(sc, [0], cam)
    assert p["valid"][0]
    th = 1 / (1 + math.exp(-float(np.float32(1.3))))
    assert abs(p["theta"][0] - th) < 1e-15 and abs(p["log_theta"][0] - math.log(th)) < 1e-15


def test_radius_bound_is_exact():
    """Beyond the pruning radius alpha < 1/255 even for theta = 1: the radius
    constant must be at least sqrt(2 ln 255) (3.3290 is not)."""
    assert project.RADIUS_K >= math.sqrt(2 * math.log(255.0))
    assert 3.3290 < math.sqrt(2 * math.log(255.0))
    for lam in (0.3, 2.0, 17.5, 1e4):
        r = project.RADIUS_K * math.sqrt(lam)            # before the ceil: the tightest case
        alpha = math.exp(-0.5 * r * r / lam)             # along the major axis, theta = 1
        assert alpha < 1 / 255
