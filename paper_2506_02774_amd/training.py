"""Differentiable rendering for training (torch.autograd over the C ABI).

`Renderer` renders a hierarchy whose Gaussian parameters are torch tensors:
the first call uploads the tree and the parameters (vy_scene_upload), later
calls repack only the parameters (vy_scene_update_gaussians) over the same
tree; the LoD cut is computed when the camera changes (it depends on the
tree's boxes only), and each call renders with the state the backward pass
needs; `GaussianRenderFn.backward` calls vy_render_backward. The loss used for
training is L1 + 0.2 (1 - SSIM), SSIM as in Wang et al. (2004) with an 11x11
Gaussian window of standard deviation 1.5 (the same definition as
`paper_2506_02774_amd.quality.ssim`, written with torch operations so that it
is differentiable).

The tree (parent, children, AABBs) stays fixed: the boxes are those given at
construction, so a cut at tau = 0 (every visible leaf) is the usual setting
for training the leaves.
"""
from __future__ import annotations

import torch

from . import (VY_ERR_STATE, RenderContext, Scene, VoyagerError, check, make_camera, vy_lod_cut, vy_render,
               vy_render_backward)

PARAMS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


class GaussianRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, sh, renderer, cam):
        params = dict(mean=mean, log_scale=log_scale, quat=quat, opacity_logit=opacity_logit, sh=sh)
        image = renderer._render(params, cam)
        ctx.renderer, ctx.cam = renderer, cam
        ctx.generation = renderer.generation
        ctx.save_for_backward(quat)
        return image

    @staticmethod
    def backward(ctx, dimage):
        (quat,) = ctx.saved_tensors
        r = ctx.renderer
        # the renderer keeps the saved state of its latest forward only
        if r.generation != ctx.generation:
            raise VoyagerError(VY_ERR_STATE, "GaussianRenderFn.backward: the renderer has rendered again since this "
                                             "forward (one forward per backward on a Renderer)")
        g = vy_render_backward(r.scene, r.cut, ctx.cam, r.ctx, dimage.contiguous(), quat_raw=quat.detach())
        return g["mean"], g["log_scale"], g["quat"], g["opacity_logit"], g["sh"], None, None


class Renderer:
    """Differentiable renderer over a fixed tree (scenegen.Scene-like host object)."""

    def __init__(self, host_tree, width, height, tau=0.0, alpha_filter=True, bg=(0.0, 0.0, 0.0),
                 max_pairs=1 << 22, device="cuda"):
        n = int(host_tree.parent.shape[0])
        t = lambda a, dt: torch.as_tensor(a, dtype=dt).to(device).contiguous()   # noqa: E731
        self.tree = dict(parent=t(host_tree.parent, torch.int32), first_child=t(host_tree.first_child, torch.int32),
                         child_count=t(host_tree.child_count, torch.int32),
                         aabb_lo=t(host_tree.aabb_lo, torch.float32), aabb_hi=t(host_tree.aabb_hi, torch.float32))
        self.n, self.tau, self.alpha_filter, self.bg = n, float(tau), bool(alpha_filter), tuple(bg)
        self.ctx = RenderContext(n, width, height, max_pairs)
        self.scene = self.cut = None
        self._cut_key = None         # the camera the cut was computed for
        self.generation = 0          # forwards rendered so far; backward differentiates the latest only

    def parameters_from(self, host_tree, device="cuda"):
        """Leaf tensors (requires_grad) initialised from a host tree's arrays."""
        out = {}
        for k in PARAMS:
            a = torch.as_tensor(getattr(host_tree, k), dtype=torch.float32).to(device)
            if k == "sh":
                a = a.reshape(self.n, 16, 3)
            out[k] = a.contiguous().requires_grad_(True)
        return out

    def _render(self, params, cam):
        self.generation += 1
        p = {k: params[k].detach().contiguous() for k in PARAMS}
        if self.scene is None:
            self.scene = Scene.from_tensors(self.tree, p)
        else:
            self.scene.update_gaussians(p)
        key = bytes(make_camera(cam))
        if self.cut is None or key != self._cut_key:
            self.cut = vy_lod_cut(self.scene, cam, self.tau, out=self.cut)
            self._cut_key = key
        img = vy_render(self.scene, self.cut, cam, self.ctx, alpha_filter=self.alpha_filter, bg=self.bg,
                        save_state=True)
        rc, need, _ = self.ctx.status()
        if rc != 0:
            raise VoyagerError(rc, f"render: {need} pairs needed")
        return img

    def __call__(self, params, cam):
        return GaussianRenderFn.apply(params["mean"], params["log_scale"], params["quat"],
                                      params["opacity_logit"], params["sh"], self, cam)


def gaussian_window(size=11, sigma=1.5, dtype=torch.float32, device="cpu"):
    x = torch.arange(size, dtype=dtype, device=device) - (size - 1) / 2.0
    g = torch.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim(a, b, L=1.0):
    """Mean SSIM of images (C, H, W), differentiable (Wang et al. 2004)."""
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    C = a.shape[0]
    g = gaussian_window(dtype=a.dtype, device=a.device)
    kx = g.view(1, 1, 1, -1).repeat(C, 1, 1, 1)
    ky = g.view(1, 1, -1, 1).repeat(C, 1, 1, 1)

    def blur(x):
        return torch.nn.functional.conv2d(torch.nn.functional.conv2d(x[None], kx, groups=C), ky, groups=C)[0]

    ma, mb = blur(a), blur(b)
    saa = blur(a * a) - ma * ma
    sbb = blur(b * b) - mb * mb
    sab = blur(a * b) - ma * mb
    m = ((2 * ma * mb + c1) * (2 * sab + c2)) / ((ma * ma + mb * mb + c1) * (saa + sbb + c2))
    return m.mean()


def loss_l1_ssim(image, target, weight=0.2):
    """L1 + weight * (1 - SSIM)."""
    return (image - target).abs().mean() + weight * (1.0 - ssim(image, target))
