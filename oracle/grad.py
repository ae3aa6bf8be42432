"""Oracle: gradients of the rendered image (FP64). Test infrastructure only.

The gradient of L = sum(w * image) with respect to the parameters of the cut's
Gaussians - world means, log-scales, quaternions (as given, before their
normalisation), opacity logits and SH coefficients - for the image that
oracle.render computes from oracle.project's projection (Section 3.1
"Culling & Projection" and "Rasterization", Eq. 3). The blend's discrete
decisions (the depth order, the candidate boxes, alpha >= alpha*, the stop
before T falls below 1e-4, the clamps alpha <= 0.99 and rho <= 0, the
Jacobian's clamped ratios and the [0, 1] colour clamp) are held at their FP64
values: the image is smooth in the parameters away from those boundaries and
this is its derivative there.

It is computed by reverse-mode automatic differentiation (torch, float64, on
the CPU) of a transcription of the projection and of the per-pixel
front-to-back blend, written with torch tensors instead of numpy arrays; the
arithmetic follows oracle.project and oracle.render step by step, and
tests/test_oracle_grad.py pins it to central finite differences of
oracle.render's numpy image and to closed forms.
"""
from __future__ import annotations

import math

import numpy as np

from . import project as _proj
from . import render as _render
from . import sh as _sh

PARAMS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def _torch():
    import torch
    return torch


def _rotation(q):
    """Rotation matrices (n, 3, 3) from quaternions (w, x, y, z), normalised here."""
    torch = _torch()
    q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    rows = [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
            2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
            2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]
    return torch.stack(rows, dim=1).reshape(-1, 3, 3)


def _sh_basis(d):
    """The degree-3 real basis of oracle.sh.basis, for unit vectors d (n, 3)."""
    torch = _torch()
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    xx, yy, zz = x * x, y * y, z * z
    r2 = xx + yy + zz
    s = _sh
    cols = [torch.full_like(x, s.C0), s.C1 * y, s.C1 * z, s.C1 * x,
            s.C2_xy * x * y, s.C2_xy * y * z, s.C2_0 * (3.0 * zz - r2), s.C2_xy * x * z, s.C2_2 * (xx - yy),
            s.C3_3 * y * (3.0 * xx - yy), s.C3_2m * x * y * z, s.C3_1 * y * (5.0 * zz - r2),
            s.C3_0 * z * (5.0 * zz - 3.0 * r2), s.C3_1 * x * (5.0 * zz - r2), s.C3_2p * z * (xx - yy),
            s.C3_3 * x * (xx - 3.0 * yy)]
    return torch.stack(cols, dim=1)


def project_torch(p, cam, dtype=None):
    """oracle.project's projection of the Gaussians whose parameters are the
    float64 tensors p[k] (k in PARAMS), differentiable. Returns a dict of
    tensors: mean2d (n, 2), conic (n, 3) = (a, b, c) of Sigma2^-1, theta,
    rgb (n, 3), and the no-grad depth, validity and pruning radius."""
    torch = _torch()
    dtype = p["mean"].dtype if dtype is None else dtype
    R = torch.as_tensor(np.asarray(cam.R, np.float64)).to(dtype)
    pos = torch.as_tensor(np.asarray(cam.pos, np.float64)).to(dtype)
    fx, fy, cx, cy, near = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy, cam.near))
    W, H = float(cam.width), float(cam.height)
    rel = p["mean"] - pos
    xc = rel @ R.T
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    valid = (z > near).detach()
    zs = torch.where(valid, z, torch.ones_like(z))
    s = torch.exp(p["log_scale"])
    M = _rotation(p["quat"]) * s[:, None, :]          # Rq diag(s)
    S3 = M @ M.transpose(1, 2)
    u = torch.clamp(x / zs, -_proj.CLAMP * cx / fx, _proj.CLAMP * (W - cx) / fx)
    v = torch.clamp(y / zs, -_proj.CLAMP * cy / fy, _proj.CLAMP * (H - cy) / fy)
    zero = torch.zeros_like(zs)
    J = torch.stack([torch.stack([fx / zs, zero, -fx * u / zs], 1),
                     torch.stack([zero, fy / zs, -fy * v / zs], 1)], 1)
    T = J @ R
    S2 = T @ S3 @ T.transpose(1, 2)
    a = S2[:, 0, 0] + _proj.LOWPASS
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + _proj.LOWPASS
    det = a * c - b * b
    valid = valid & (det > 0).detach()
    dets = torch.where(valid, det, torch.ones_like(det))
    conic = torch.stack([c / dets, -b / dets, a / dets], 1)
    mean2d = torch.stack([fx * x / zs + cx, fy * y / zs + cy], 1)
    with torch.no_grad():
        mid = 0.5 * (a + c)
        lam = mid + torch.sqrt(torch.clamp(mid * mid - dets, min=0.0))
        radius = torch.ceil(_proj.RADIUS_K * torch.sqrt(lam))
    theta = torch.sigmoid(p["opacity_logit"])
    d = rel / torch.linalg.norm(rel, dim=1, keepdim=True)
    col = torch.einsum("nk,nkc->nc", _sh_basis(d), p["sh"]) + 0.5
    rgb = torch.clamp(col, 0.0, 1.0)
    return dict(mean2d=mean2d, conic=conic, theta=theta, rgb=rgb, depth=z.detach(), valid=valid, radius=radius)


def blend_torch(pr, ids, px, py, bg):
    """oracle.render.render_pixels' blend of pixels (px, py) over the
    projected Gaussians pr (tensors from project_torch), differentiable in
    the projected attributes. Returns rgb (P, 3)."""
    torch = _torch()
    depth = pr["depth"].numpy()
    v = np.nonzero(pr["valid"].numpy())[0]
    order = v[np.lexsort((np.asarray(ids)[v], depth[v]))]
    dt = pr["mean2d"].dtype
    cxp = torch.as_tensor(np.asarray(px, np.float64) + 0.5).to(dt)
    cyp = torch.as_tensor(np.asarray(py, np.float64) + 0.5).to(dt)
    o = torch.as_tensor(order)
    m = pr["mean2d"][o]
    r = pr["radius"][o] + _render.SLACK
    with torch.no_grad():
        keep = ((m[:, 0] + r >= cxp.min()) & (m[:, 0] - r <= cxp.max()) &
                (m[:, 1] + r >= cyp.min()) & (m[:, 1] - r <= cyp.max()))
    k = torch.nonzero(keep)[:, 0]
    cand = o[k]
    mc, rc = m[k], r[k]
    con = pr["conic"][cand]
    th = pr["theta"][cand]
    rgb = pr["rgb"][cand]
    dx = cxp[:, None] - mc[None, :, 0]
    dy = cyp[:, None] - mc[None, :, 1]
    with torch.no_grad():
        inside = (dx.abs() <= rc[None, :]) & (dy.abs() <= rc[None, :])
    Q = con[None, :, 0] * dx * dx + 2.0 * con[None, :, 1] * dx * dy + con[None, :, 2] * dy * dy
    rho = torch.clamp(-0.5 * Q, max=0.0)
    alpha = torch.clamp(th[None, :] * torch.exp(rho), max=_render.ALPHA_MAX)
    alpha = torch.where(inside, alpha, torch.zeros_like(alpha))
    with torch.no_grad():
        use = inside & (alpha >= _render.ALPHA_MIN)
    a = torch.where(use, alpha, torch.zeros_like(alpha))
    Tafter = torch.cumprod(1.0 - a, dim=1)
    ones = torch.ones((len(px), 1), dtype=Tafter.dtype)
    Tbefore = torch.cat([ones, Tafter[:, :-1]], dim=1)
    with torch.no_grad():
        stop = Tafter < _render.T_MIN                  # monotone along the row
        first_stop = stop & ~torch.cat([torch.zeros((len(px), 1), dtype=torch.bool), stop[:, :-1]], dim=1)
        active = use & ~stop
        any_stop = stop.any(dim=1)
    w = torch.where(active, a * Tbefore, torch.zeros_like(a))
    C = w @ rgb
    T_stop = torch.where(first_stop, Tbefore, torch.zeros_like(Tbefore)).sum(dim=1)
    T = torch.where(any_stop, T_stop, Tafter[:, -1] if a.shape[1] else torch.ones(len(px), dtype=a.dtype))
    return C + T[:, None] * torch.as_tensor(np.asarray(bg, np.float64)).to(dt)[None, :]


def image_and_grads(scene, ids, cam, dL_dimage, bg=(0.0, 0.0, 0.0), tile=16, dtype="float64"):
    """Image (3, H, W) of the Gaussians `ids` of `scene` seen by `cam`, and the
    gradients of sum(dL_dimage * image) with respect to their parameters,
    as float64 numpy arrays indexed like `ids` (quat: the stored, unnormalised
    quaternion). The image is blended tile by tile (16x16 pixels); each
    tile's contribution is differentiated in turn and accumulated. `dtype`
    "float32" evaluates the same steps in float32 (to see how far float32
    rounding alone moves each gradient); results are returned as float64."""
    torch = _torch()
    tdt = getattr(torch, dtype)
    ids = np.asarray(ids, np.int64)
    shp = dict(mean=(len(ids), 3), log_scale=(len(ids), 3), quat=(len(ids), 4), opacity_logit=(len(ids),),
               sh=(len(ids), 16, 3))
    p = {k: torch.tensor(np.asarray(getattr(scene, k))[ids].astype(np.float64).reshape(shp[k])).to(tdt)
         .requires_grad_(True) for k in PARAMS}
    pr = project_torch(p, cam)
    diff = {k: pr[k] for k in ("mean2d", "conic", "theta", "rgb")}
    leaves = {k: t.detach().requires_grad_(True) for k, t in diff.items()}
    pr_leaf = dict(pr, **leaves)
    W, H = cam.width, cam.height
    wimg = np.asarray(dL_dimage, np.float64)
    img = np.zeros((3, H, W))
    acc = {k: torch.zeros_like(t) for k, t in leaves.items()}
    tx_n, ty_n = (W + tile - 1) // tile, (H + tile - 1) // tile
    for t in range(tx_n * ty_n):
        ty, tx = divmod(t, tx_n)
        xs = np.arange(tx * tile, min(W, (tx + 1) * tile))
        ys = np.arange(ty * tile, min(H, (ty + 1) * tile))
        PX, PY = np.meshgrid(xs, ys)
        PX, PY = PX.ravel(), PY.ravel()
        C = blend_torch(pr_leaf, ids, PX, PY, bg)
        img[:, PY, PX] = C.detach().numpy().T
        g = torch.as_tensor(wimg[:, PY, PX].T).to(tdt)
        loss = (C * g).sum()
        if loss.requires_grad:
            gr = torch.autograd.grad(loss, list(leaves.values()), allow_unused=True)
            for (k, _), gk in zip(leaves.items(), gr):
                if gk is not None:
                    acc[k] += gk
    torch.autograd.backward([diff[k] for k in leaves], [acc[k] for k in leaves])
    grads = {k: (p[k].grad.double().numpy().copy() if p[k].grad is not None else np.zeros(shp[k])) for k in PARAMS}
    grads["sh"] = grads["sh"].reshape(len(ids), 48)
    return img, grads
