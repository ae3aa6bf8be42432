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


def _iso_cov2d(f, z, sigma, u, v):
    """Sigma2 of an isotropic Gaussian (Sigma3 = sigma^2 I) seen by an unrotated
    pinhole, written out by hand: J = (f/z) [[1, 0, -u], [0, 1, -v]], so
    J J^T = (f/z)^2 [[1 + u^2, u v], [u v, 1 + v^2]], plus the 0.3 low-pass."""
    k = (f / z) ** 2 * sigma * sigma
    return np.array([k * (1 + u * u) + 0.3, k * u * v, k * (1 + v * v) + 0.3])


def test_jacobian_clamp_off_axis():
    """Past 1.3x the half-extent of the image (in x/z or y/z) the Jacobian
    takes the clamped ratio while mean2D keeps the true one (3DGS EWA
    convention, Section 3.1 "Culling & Projection"). A 256x128 image has
    different horizontal and vertical bounds (1.3 cx / fx and 1.3 cy / fy)."""
    cam = scenegen.identity_camera(256, 128)
    f = float(np.float32(cam.fx))
    ub, vb = 1.3 * 128.0 / f, 1.3 * 64.0 / f          # 0.7506 and 0.3753
    z = 10.0
    cases = [  # (x, y) in camera space; the ratios x/z, y/z the Jacobian must use
        ((12.0, 1.0), (ub, 0.1)),        # right of the bound
        ((-12.0, 1.0), (-ub, 0.1)),      # left of it
        ((2.0, 6.0), (0.2, vb)),         # below the vertical bound (+y is down)
        ((2.0, -6.0), (0.2, -vb)),       # above it
        ((-15.0, -9.0), (-ub, -vb)),     # both clamped
        ((7.0, 3.5), (0.7, 0.35)),       # just inside both bounds: unclamped
    ]
    for (x, y), (u, v) in cases:
        sc = _one([x, y, z], [math.log(0.5)] * 3)
        sigma = math.exp(float(sc.log_scale[0, 0]))
        p = project.project(sc, [0], cam)
        np.testing.assert_allclose(p["cov2d"][0], _iso_cov2d(f, z, sigma, u, v), rtol=1e-9, atol=1e-9)
        # the mean is not clamped
        np.testing.assert_allclose(p["mean2d"][0], [f * x / z + 128.0, f * y / z + 64.0], rtol=1e-12)


def test_sh_view_direction_is_world_mean_minus_camera():
    """The SH colour is evaluated at the unit vector from the camera centre to
    the mean, in world axes. With one degree-1 coefficient c set per channel
    (Y_1,-1 = C1 y, Y_1,0 = C1 z, Y_1,1 = C1 x, C1 = 0.4886025119...), the
    colour is 0.5 + C1 c d_k; a reversed direction or camera-frame axes give
    other values. The camera is rotated (heading 0.7 rad, pitch -0.2 rad) and
    off the origin."""
    C1 = 0.48860251190291992
    cam = scenegen.look_camera([10.0, -5.0, 1.7], 0.7, -0.2, 128, 96)
    pos = cam.pos.astype(np.float64)
    fwd = cam.R[2].astype(np.float64)
    right = cam.R[0].astype(np.float64)
    down = cam.R[1].astype(np.float64)
    sh = np.zeros((16, 3), np.float32)
    sh[2, 0] = 0.6      # red follows d_z
    sh[3, 1] = -0.7     # green follows d_x
    sh[1, 2] = 0.8      # blue follows d_y
    for off in ([0.0, 0.0], [1.5, -0.8], [-2.0, 1.0]):     # on the optical axis, then off it
        mu = (pos + 6.0 * fwd + off[0] * right + off[1] * down).astype(np.float32)
        sc = scenegen.tree_from_arrays([-1], [-1], [0], [[0, 0, 0]], [[0, 0, 0]], mean=[mu], sh=[sh])
        p = project.project(sc, [0], cam)
        d = mu.astype(np.float64) - pos
        d /= np.linalg.norm(d)
        c = sh.astype(np.float64)
        want = 0.5 + C1 * np.array([c[2, 0] * d[2], c[3, 1] * d[0], c[1, 2] * d[1]])
        assert np.all((want > 0.05) & (want < 0.95))          # away from the [0, 1] clamp
        np.testing.assert_allclose(p["rgb"][0], want, rtol=0, atol=1e-12)
