"""Oracle: EWA culling & projection of cut Gaussians (FP64). Test infrastructure only.

Section 3.1 "Culling & Projection": the selected Gaussians are projected onto
the image plane and those outside the view frustum are culled. The paper only
cites 3DGS for the projection; the readings (the conventional 3DGS EWA
splatting constants) are:

* view transform x_c = R (mu - pos); culled when z_c <= near (0.2 m);
* Sigma3 = Rq diag(s^2) Rq^T with s = exp(log_scale), Rq from the unit quaternion;
* J = [[fx/z, 0, -fx u/z], [0, fy/z, -fy v/z]] where u = x/z and v = y/z are
  clamped to 1.3x the image's half-extent in normalised coordinates;
* Sigma2 = J R Sigma3 R^T J^T + 0.3 I (low-pass), conic = Sigma2^-1;
* mean2D = (fx x/z + cx, fy y/z + cy); depth = z;
* radius r = ceil(3.33 sqrt(lambda_max(Sigma2))) pixels: beyond it
  rho < -ln 255, so alpha = theta e^rho < 1/255 for any theta <= 1 (an exact
  pruning bound, not an approximation);
* theta = sigmoid(opacity logit), log theta precomputed (Section 4.2, Eq. 4);
* colour from the degree-3 SH expansion (see oracle.sh).
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh

LOWPASS = 0.3
CLAMP = 1.3
RADIUS_K = 3.33     # > sqrt(2 ln 255) = 3.329043...; 3.3290 would fall short of the bound


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices (n, 3, 3) from quaternions (n, 4) = (w, x, y, z), normalised here."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((len(q), 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def covariance3d(log_scale: np.ndarray, quat: np.ndarray) -> np.ndarray:
    s = np.exp(np.asarray(log_scale, np.float64))
    Rq = quat_to_rot(quat)
    return np.einsum("nij,nj,nkj->nik", Rq, s * s, Rq)


def project(scene, ids, cam):
    """Project Gaussians `ids` of `scene` with camera `cam`.

    Returns a dict of float64 arrays indexed like `ids`; `valid` is False for
    culled Gaussians (z <= near, or a degenerate 2D covariance)."""
    ids = np.asarray(ids, np.int64)
    R = np.asarray(cam.R, np.float64)
    pos = np.asarray(cam.pos, np.float64)
    fx, fy, cx, cy, near = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy, cam.near))
    W, H = float(cam.width), float(cam.height)
    mu = scene.mean[ids].astype(np.float64)
    # Products written as einsum sums: numpy's einsum runs its own loops,
    # never the BLAS library, which project_threaded must not enter from
    # several threads at once (numpy's threaded OpenBLAS has returned wrong
    # products to concurrent callers).
    xc = np.einsum("nj,ij->ni", mu - pos, R)     # R (mu - pos)
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    valid = z > near
    zs = np.where(valid, z, 1.0)
    S3 = covariance3d(scene.log_scale[ids], scene.quat[ids])
    u = np.clip(x / zs, -CLAMP * cx / fx, CLAMP * (W - cx) / fx)
    v = np.clip(y / zs, -CLAMP * cy / fy, CLAMP * (H - cy) / fy)
    n = len(ids)
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = fx / zs
    J[:, 0, 2] = -fx * u / zs
    J[:, 1, 1] = fy / zs
    J[:, 1, 2] = -fy * v / zs
    T = np.einsum("nij,jk->nik", J, R)            # J R
    S2 = np.einsum("nik,nlk->nil", np.einsum("nij,njk->nik", T, S3), T)   # (T S3) T^T
    a = S2[:, 0, 0] + LOWPASS
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + LOWPASS
    det = a * c - b * b
    valid &= det > 0
    dets = np.where(det > 0, det, 1.0)
    conic = np.stack([c / dets, -b / dets, a / dets], axis=1)
    mx = fx * x / zs + cx
    my = fy * y / zs + cy
    mid = 0.5 * (a + c)
    lam = mid + np.sqrt(np.maximum(0.0, mid * mid - dets))
    radius = np.ceil(RADIUS_K * np.sqrt(lam))
    lg = scene.opacity_logit[ids].astype(np.float64)
    theta = 1.0 / (1.0 + np.exp(-lg))
    log_theta = -np.log1p(np.exp(-lg))
    rgb = _sh.colour(scene.sh[ids], mu - pos)
    return dict(ids=ids, valid=valid, mean2d=np.stack([mx, my], 1), conic=conic, cov2d=np.stack([a, b, c], 1),
                depth=z, radius=radius, lambda_max=lam, theta=theta, log_theta=log_theta, rgb=rgb,
                near_margin=np.abs(z - near) / np.maximum(np.abs(z), near))


def project_threaded(scene, ids, cam, threads: int = 1, chunk: int = 1 << 18):
    """project() of `ids` in chunks on `threads` threads (numpy releases the
    GIL in its array loops); the per-Gaussian arithmetic is project()'s."""
    ids = np.asarray(ids, np.int64)
    if threads <= 1 or len(ids) <= chunk:
        return project(scene, ids, cam)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda a: project(scene, ids[a:a + chunk], cam), range(0, len(ids), chunk)))
    return {k: np.concatenate([q[k] for q in parts]) for k in parts[0]}
