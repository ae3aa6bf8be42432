"""GPU checks of vy_render_backward (through the C ABI): the gradients of
sum(w * image) for random weights w, with respect to means, log-scales,
quaternions, opacity logits and SH coefficients, against central finite
differences of the FP64 oracle's image along random directions (relative
error <= 1e-3), with the oracle confirming that no step flipped a blend
decision (alpha*, transmittance stop); filtered and unfiltered frames give the
same gradients; the saved-state preconditions are enforced."""
import dataclasses
import math

import numpy as np
import pytest

import scenegen
from oracle import project as oproj, render as orender

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

W, H = 64, 64
BG = (0.1, 0.2, 0.3)
GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


@pytest.fixture(scope="module")
def world():
    vy = require_gpu()
    import torch
    leaves = scenegen.random_gaussians(2000, 21, W, H, depth_range=(2.0, 20.0), scale_range=(-3.0, -0.7))
    host = scenegen.build_hierarchy(dict(mean=leaves.mean, log_scale=leaves.log_scale, quat=leaves.quat,
                                         opacity_logit=leaves.opacity_logit, sh=leaves.sh))
    cam = scenegen.identity_camera(W, H)
    th = 0.1
    Rz = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    cam.R = (Rz @ np.asarray(cam.R, np.float64)).astype(np.float32)
    cam.pos = np.array([0.1, -0.05, 0.2], np.float32)
    sc = vy.Scene(host)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 20)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    F, C = cut.ids()
    assert np.all(host.child_count[C] == 0) and len(C) > 1500
    w = np.random.default_rng(3).standard_normal((3, H, W))
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    qraw = torch.from_numpy(host.quat).cuda()
    return vy, torch, host, sc, ctx, cut, C, cam, w, wt, qraw


def _grads(world, filt):
    vy, torch, host, sc, ctx, cut, C, cam, w, wt, qraw = world
    vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, bg=BG, save_state=True)
    vy.check(ctx.status()[0])
    g = vy.vy_render_backward(sc, cut, cam, ctx, wt, quat_raw=qraw, mean2d=True)
    return {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}


def _oracle_loss(world, P):
    vy, torch, host, sc, ctx, cut, C, cam, w, wt, qraw = world
    s = dataclasses.replace(host, **P)
    r = orender.render_image(oproj.project(s, C, cam), W, H, bg=BG, signature=True)
    return float((w * r["image"]).sum()), r["signature"]


def test_gradients_match_oracle_finite_differences(world):
    vy, torch, host, sc, ctx, cut, C, cam, w, wt, qraw = world
    G = _grads(world, True)
    G["sh"] = G["sh"].reshape(-1, 16, 3)
    P0 = {k: getattr(host, k).astype(np.float64) for k in GROUPS}
    L0, sig0 = _oracle_loss(world, P0)
    # the GPU image and the oracle's agree, so the loss they differentiate is the same
    img = vy.vy_render(sc, cut, cam, ctx, alpha_filter=True, bg=BG).cpu().numpy()
    assert abs(float((w * img).sum()) - L0) <= 1e-3 * abs(L0) + 1e-2
    # Gaussians that reach the image
    live = [int(i) for i in C if any(np.abs(G[k][i]).max() > 0 for k in GROUPS)]
    assert len(live) > 500
    rng = np.random.default_rng(7)
    checked = 0
    for group in GROUPS + ("all",):
        ok_dirs = 0
        for trial in range(6):
            if ok_dirs == 2:
                break
            sub = rng.choice(live, 16, replace=False)
            D = {k: np.zeros_like(v) for k, v in P0.items()}
            for k in GROUPS:
                if group in (k, "all"):
                    D[k][sub] = rng.standard_normal(D[k][sub].shape)
            h = 1e-6
            Lp, sp = _oracle_loss(world, {k: P0[k] + h * D[k] for k in GROUPS})
            Lm, sm = _oracle_loss(world, {k: P0[k] - h * D[k] for k in GROUPS})
            if np.any(sp != sig0) or np.any(sm != sig0):
                continue                      # a blend decision flipped within the step: not differentiable here
            fd = (Lp - Lm) / (2 * h)
            ad = sum(float((G[k] * D[k]).sum()) for k in GROUPS)
            # relative to the derivative, or to its terms' size where they cancel
            scale = max(abs(fd), abs(ad), 1e-2 * sum(float(np.abs(G[k] * D[k]).sum()) for k in GROUPS), 1e-6)
            rel = abs(fd - ad) / scale
            print(f"{group:14s} fd {fd: .6e} gpu {ad: .6e} rel {rel:.2e}", flush=True)
            assert rel <= 1e-3, (group, fd, ad)
            ok_dirs += 1
            checked += 1
        assert ok_dirs == 2, group
    assert checked == 12


def test_filtered_and_unfiltered_give_the_same_gradients(world):
    a = _grads(world, True)
    b = _grads(world, False)
    for k in a:
        scale = max(1e-6, float(np.abs(a[k]).max()))
        assert np.abs(a[k] - b[k]).max() <= 1e-5 * scale, k


def test_backward_preconditions(world):
    vy, torch, host, sc, ctx, cut, C, cam, w, wt, qraw = world
    vy.vy_render(sc, cut, cam, ctx, bg=BG)                                 # without save_state
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_render_backward(sc, cut, cam, ctx, wt)
    assert e.value.code == vy.VY_ERR_STATE
    vy.vy_render(sc, cut, cam, ctx, bg=BG, save_state=True)
    other = scenegen.identity_camera(W, H)
    with pytest.raises(vy.VoyagerError) as e:                              # another camera
        vy.vy_render_backward(sc, cut, other, ctx, wt)
    assert e.value.code == vy.VY_ERR_STATE
    vy.vy_lod_cut(sc, cam, 0.0, prev=cut, out=cut)                         # the cut was recomputed
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_render_backward(sc, cut, cam, ctx, wt)
    assert e.value.code == vy.VY_ERR_STATE
    vy.vy_render(sc, cut, cam, ctx, bg=BG, save_state=True, lut_entries=32)   # LUT: no backward
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_render_backward(sc, cut, cam, ctx, wt)
    assert e.value.code == vy.VY_ERR_STATE
