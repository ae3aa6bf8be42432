"""GPU checks of vy_render_backward (through the C ABI): the gradients of
sum(w * image) for random weights w, with respect to means, log-scales,
quaternions, opacity logits and SH coefficients, element by element against
the FP64 oracle gradient (relative error <= 1e-3), including Gaussians under
the Jacobian clamp and a tile of more than 4096 pairs; against central finite
differences of the FP64 oracle's image along random directions over
Gaussians the oracle sees reaching the image (relative error <= 1e-3), with
the oracle confirming that no step flipped a blend decision (alpha*,
transmittance stop); filtered and unfiltered frames give the same gradients;
the saved-state preconditions are enforced."""
import dataclasses
import math

import numpy as np
import pytest

import scenegen
from oracle import grad as ograd, project as oproj, render as orender

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

W, H = 64, 64
BG = (0.1, 0.2, 0.3)
GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def _leaves():
    """2000 Gaussians spread over the view, 16 large ones off to the sides past
    the Jacobian clamp (1.3x the half-extent) whose footprints reach the image,
    and a cluster of 4800 faint small ones inside one tile (more than 4096
    pairs there: blended band by band by waves of their own)."""
    a = scenegen.random_gaussians(2000, 21, W, H, depth_range=(2.0, 20.0), scale_range=(-3.0, -0.7))
    rng = np.random.default_rng(22)
    f = (W / 2.0) / math.tan(math.radians(30.0))
    n = 16
    z = rng.uniform(3.0, 8.0, n)
    u = rng.choice([-1.0, 1.0], n) * rng.uniform(0.85, 1.1, n)
    clamp = np.stack([u * z, rng.uniform(-0.4, 0.4, n) * z, z], 1)
    m = 4800
    zc = rng.uniform(4.0, 16.0, m)
    px = rng.uniform(19.0, 29.0, m)            # tile (1, 1) spans pixels 16..31
    py = rng.uniform(19.0, 29.0, m)
    clus = np.stack([(px - W / 2) * zc / f, (py - H / 2) * zc / f, zc], 1)
    mean = np.concatenate([a.mean, clamp, clus]).astype(np.float32)
    ls = np.concatenate([a.log_scale, rng.uniform(-0.6, -0.2, (n, 3)),
                         np.log(0.02 * zc / 10)[:, None] + rng.uniform(-0.2, 0.2, (m, 3))]).astype(np.float32)
    q = np.concatenate([a.quat, rng.normal(size=(n + m, 4))]).astype(np.float32)
    lg = np.concatenate([a.opacity_logit, rng.normal(0, 1.0, n), rng.normal(-5.0, 0.3, m)]).astype(np.float32)
    sh = np.concatenate([a.sh, rng.normal(0, 0.2, (n + m, 16, 3))]).astype(np.float32)
    sh[2000:, 0] += 0.5
    return dict(mean=mean, log_scale=ls, quat=q, opacity_logit=lg, sh=sh)


@pytest.fixture(scope="module")
def world():
    vy = require_gpu()
    import torch
    host = scenegen.build_hierarchy(_leaves())
    cam = scenegen.identity_camera(W, H)
    th = 0.1
    Rz = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    cam.R = (Rz @ np.asarray(cam.R, np.float64)).astype(np.float32)
    cam.pos = np.array([0.1, -0.05, 0.2], np.float32)
    sc = vy.Scene(host)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 20)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    F, C = cut.ids()
    assert np.all(host.child_count[C] == 0) and len(C) > 6000
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
    # Gaussians that reach the image, as the oracle sees them (its FP64 gradient is non-zero)
    _, OG = ograd.image_and_grads(host, C, cam, w, bg=BG)
    live = [int(C[j]) for j in range(len(C)) if any(np.abs(OG[k][j]).max() > 0 for k in GROUPS)]
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


def test_gradients_match_oracle_element_by_element(world):
    """Every parameter of every Gaussian of the cut against the FP64 oracle
    gradient (oracle.grad). The bar per element: relative error <= 1e-3,
    against the element itself or, where it is a sum of terms that cancel,
    against 1e-2 of the largest gradient of the same Gaussian and parameter
    group. Where float32 rounding alone moves an element by more (the same
    definition evaluated in float32 by the oracle: reach r = the largest
    float32 error in that Gaussian's group), the GPU must stay within 16 r,
    and such elements must be under 0.1 % of all. Gaussians with no oracle
    gradient get none on the GPU. The scene includes Gaussians under the
    Jacobian clamp and a tile of more than 4096 pairs (band jobs), whose
    faint Gaussians blend behind thousands of others."""
    vy, torch, host, sc, ctx, cut, C, cam, w, wt, qraw = world
    G = _grads(world, True)
    keys, vals, ranges = ctx.pairs(W, H)
    length = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    assert length.max() > 4096, length.max()
    img, OG = ograd.image_and_grads(host, C, cam, w, bg=BG)
    _, O32 = ograd.image_and_grads(host, C, cam, w, bg=BG, dtype="float32")
    gimg = vy.vy_render(sc, cut, cam, ctx, alpha_filter=True, bg=BG).cpu().numpy()
    assert np.abs(gimg - img).max() < 2e-3
    p = oproj.project(host, C, cam)
    f = float(np.float32(cam.fx))
    u = (p["mean2d"][:, 0] - cam.cx) / f
    under_clamp = p["valid"] & (np.abs(u) > 1.3 * cam.cx / f)
    heavy_tile = int(np.argmax(length))
    in_heavy = np.zeros(len(C), bool)
    in_heavy[np.unique(vals[ranges[heavy_tile, 0]:ranges[heavy_tile, 1]])] = True
    worst, n_el, n_f32 = {}, 0, 0
    for k in GROUPS:
        o = OG[k].reshape(len(C), -1)
        g = G[k][C].reshape(len(C), -1)
        gmax = np.abs(o).max(axis=1, keepdims=True)
        live = gmax[:, 0] > 0
        assert np.all(g[~live] == 0), k                 # no oracle gradient: none on the GPU either
        err = np.abs(g - o)
        rel = err / np.maximum(np.maximum(np.abs(o), 1e-2 * gmax), 1e-300)
        reach = np.abs(O32[k].reshape(len(C), -1) - o).max(axis=1, keepdims=True)
        strict = rel <= 1e-3
        by_f32 = ~strict & (err <= 16 * reach)
        bad = live[:, None] & ~strict & ~by_f32
        assert not bad.any(), (k, np.argwhere(bad)[:5].tolist(), float(rel[bad].max()))
        n_el += int(live.sum()) * o.shape[1]
        n_f32 += int((by_f32 & live[:, None]).sum())
        worst[k] = float(rel[live][strict[live]].max())
        for name, sel in (("clamp", under_clamp), ("heavy", in_heavy)):
            m = (sel & live)[:, None] & strict
            if m.any():
                worst[f"{k}/{name}"] = float(rel[m].max())
    print(f"{n_el} elements, {n_f32} within 16x their float32 reach; {int(under_clamp.sum())} Gaussians under the "
          f"clamp, {int(in_heavy.sum())} in the {int(length.max())}-pair tile; worst rel (elements at 1e-3) " +
          ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    assert n_f32 <= 1e-3 * n_el
    assert int((under_clamp & (np.abs(OG["mean"]).max(axis=1) > 0)).sum()) >= 4
    assert int((in_heavy & (np.abs(OG["sh"]).max(axis=1) > 0)).sum()) >= 500


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
