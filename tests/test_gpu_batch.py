"""GPU checks of batched rendering (vy_render_batch, through the C ABI):
frames of several viewers, over different scenes and resolutions, rendered
with one launch per stage are each bitwise the image vy_render writes for
that viewer alone, with and without the preemptive filter and for every walk,
including a view whose tiles hold more than 4096 pairs (band jobs); the batch
counts are the sums of the frames'; and bad batches are refused."""
import numpy as np
import pytest

import scenegen

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world(tiny_scene, tiny_cams):
    vy = require_gpu()
    import torch
    # a 200k-leaf city (the full-scale recipe at a smaller extent), its walkthrough
    cfg = scenegen.scaled_config("full", 200_000)
    city = scenegen.make_city(cfg)
    city_cams = scenegen.walkthrough(cfg, frames=12)
    # a heavy view: 60k small Gaussians in a 64x48 image (tiles of more than 4096 pairs)
    leaves = scenegen.random_gaussians(60000, 11, 64, 48, depth_range=(1.0, 60.0), scale_range=(-4.0, -1.0))
    heavy = scenegen.build_hierarchy(dict(mean=leaves.mean, log_scale=leaves.log_scale, quat=leaves.quat,
                                          opacity_logit=leaves.opacity_logit, sh=leaves.sh))
    scenes = dict(tiny=vy.Scene(tiny_scene), city=vy.Scene(city), heavy=vy.Scene(heavy))

    views = [
        ("tiny", tiny_cams[3], 2.0),
        ("city", _resized(city_cams[5], 640, 360), 2.0),
        ("tiny", _resized(tiny_cams[6], 96, 64), 1.0),
        ("heavy", scenegen.identity_camera(64, 48), 0.0),
        ("city", _resized(city_cams[11], 1280, 720), 2.0),
        ("city", _resized(city_cams[2], 200, 120), 4.0),
    ]
    cuts = []
    for name, cam, tau in views:
        cuts.append(vy.vy_lod_cut(scenes[name], cam, tau))
    return vy, torch, scenes, views, cuts


def _resized(cam, w, h):
    import math
    yaw = math.atan2(float(cam.R[2][1]), float(cam.R[2][0]))
    return scenegen.look_camera(cam.pos, yaw, 0.0, w, h)


def _alone(vy, torch, scenes, views, cuts, filt, walk):
    out, pairs, vis = [], 0, 0
    for (name, cam, tau), cut in zip(views, cuts):
        sc = scenes[name]
        ctx = vy.RenderContext(sc.n, cam.width, cam.height, 1 << 22)
        out.append(vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, walk=walk, bg=(0.1, 0.2, 0.3)))
        rc, p, v = ctx.status()
        vy.check(rc)
        pairs += p
        vis += v
    return out, pairs, vis


@pytest.mark.parametrize("filt", [False, True])
@pytest.mark.parametrize("walk", [0, 1, 2])
def test_batch_equals_frames_alone(world, filt, walk):
    vy, torch, scenes, views, cuts = world
    ref, pairs, vis = _alone(vy, torch, scenes, views, cuts, filt, walk)
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for _, c, _ in views)
    ctx = vy.BatchContext(8, 1 << 21, tiles, 1 << 23)
    imgs = [torch.full((3, c.height, c.width), float("nan"), device="cuda") for _, c, _ in views]
    vy.vy_render_batch([(scenes[n], cut, c, img) for (n, c, _), cut, img in zip(views, cuts, imgs)], ctx,
                       alpha_filter=filt, walk=walk, bg=(0.1, 0.2, 0.3))
    rc, bp, bv = ctx.status()
    vy.check(rc)
    print(f"{len(views)} views, {tiles} tiles: pairs {bp} (alone {pairs}), Gaussians with pairs {bv} ({vis})",
          flush=True)
    assert (bp, bv) == (pairs, vis)
    for i, (a, b) in enumerate(zip(imgs, ref)):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (i, views[i][0])


def test_batch_has_band_job_tiles(world):
    vy, torch, scenes, views, cuts = world
    sc = scenes["heavy"]
    cam = views[3][1]
    ctx = vy.RenderContext(sc.n, cam.width, cam.height, 1 << 22)
    vy.vy_render(sc, cuts[3], cam, ctx, alpha_filter=True)
    keys, vals, ranges = ctx.pairs(cam.width, cam.height)
    assert int((ranges[:, 1] - ranges[:, 0]).max()) > 4096


def test_batch_reuse_and_refusals(world):
    vy, torch, scenes, views, cuts = world
    ctx = vy.BatchContext(4, 1 << 21, 4000, 1 << 23)
    # consecutive batches of different sizes on one context
    for sel in ([0, 2], [1], [0, 1, 2, 3]):
        ref, _, _ = _alone(vy, torch, scenes, [views[i] for i in sel], [cuts[i] for i in sel], True, 0)
        imgs = [torch.empty((3, views[i][1].height, views[i][1].width), device="cuda") for i in sel]
        vy.vy_render_batch([(scenes[views[i][0]], cuts[i], views[i][1], img) for i, img in zip(sel, imgs)], ctx,
                           alpha_filter=True, bg=(0.1, 0.2, 0.3))
        vy.check(ctx.status()[0])
        for a, b in zip(imgs, ref):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), sel
    big = [(scenes["city"], cuts[4], views[4][1], torch.empty((3, 720, 1280), device="cuda"))] * 2
    with pytest.raises(vy.VoyagerError) as e:                  # more tiles than the context holds
        vy.vy_render_batch(big, ctx)
    assert e.value.code == vy.VY_ERR_ARG
    with pytest.raises(vy.VoyagerError) as e:                  # more views than the context holds
        vy.vy_render_batch([big[0]] * 5, ctx)
    assert e.value.code == vy.VY_ERR_ARG
    fresh = vy.Cut(scenes["tiny"])
    with pytest.raises(vy.VoyagerError) as e:                  # a cut never computed
        vy.vy_render_batch([(scenes["tiny"], fresh, views[0][1], torch.empty((3, 256, 256), device="cuda"))], ctx)
    assert e.value.code == vy.VY_ERR_STATE
    with pytest.raises(vy.VoyagerError) as e:                  # a cut of another scene
        vy.vy_render_batch([(scenes["city"], cuts[0], views[0][1], torch.empty((3, 256, 256), device="cuda"))],
                           ctx)
    assert e.value.code == vy.VY_ERR_ARG
