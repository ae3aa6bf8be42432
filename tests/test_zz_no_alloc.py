"""GPU check of vy_render_noalloc (the rendering entry point that allocates
nothing: its scratch is the library's static device array), called through
the C ABI: two calls in a row, the second with a smaller input (a smaller
image of a smaller cut), each bitwise equal to vy_render with a context of
its own, and its counts equal to that context's status."""
import numpy as np
import pytest

import scenegen

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _frame(vy, torch, host, cam, tau, filt):
    """vy_render with its own context, then vy_render_noalloc on the same cut."""
    sc = vy.Scene(host)
    cut = vy.vy_lod_cut(sc, cam, tau)
    ctx = vy.RenderContext(sc.n, cam.width, cam.height, 1 << 22)
    ref = vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt)
    rc, n_pairs, n_vis = ctx.status()
    vy.check(rc, "vy_render_status")
    img = torch.full((3, cam.height, cam.width), float("nan"), device="cuda")
    counts = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    vy.vy_render_noalloc(sc, cut, cam, image=img, counts=counts, alpha_filter=filt)
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy()
    F, C = cut.ids()
    print(f"{cam.width}x{cam.height} |C| {len(C)} pairs {n_pairs} visible {n_vis} counts {cnt.tolist()}", flush=True)
    return ref, img, cnt, n_pairs, n_vis, len(C)


@pytest.mark.parametrize("filt", [True, False])
def test_noalloc_equals_vy_render_twice(tiny_scene, tiny_cams, filt):
    vy = require_gpu()
    import torch
    assert len(tiny_cams) > 5
    # first call: the tiny city at 256x256
    ref, img, cnt, n_pairs, n_vis, nc = _frame(vy, torch, tiny_scene, tiny_cams[5], 2.0, filt)
    assert n_pairs > 1000 and nc < vy.NOALLOC_MAX_GAUSSIANS and n_pairs < vy.NOALLOC_MAX_PAIRS
    assert torch.equal(img.view(torch.int32), ref.view(torch.int32))
    assert cnt.tolist() == [n_pairs, n_vis, 0, 0]
    # second call, smaller: a 4000-leaf city at 96x64 (the array keeps the first call's contents)
    cfg = scenegen.scaled_config("tiny", 4000, width=96, height=64)
    small = scenegen.make_city(cfg)
    cam = scenegen.walkthrough(cfg, frames=2, width=96, height=64)[1]
    ref2, img2, cnt2, n_pairs2, n_vis2, nc2 = _frame(vy, torch, small, cam, 2.0, filt)
    assert 0 < n_pairs2 < n_pairs and nc2 < nc
    assert torch.equal(img2.view(torch.int32), ref2.view(torch.int32))
    assert cnt2.tolist() == [n_pairs2, n_vis2, 0, 0]


def test_noalloc_refuses_sizes_beyond_the_maximum(tiny_scene, tiny_cams):
    vy = require_gpu()
    import torch
    sc = vy.Scene(tiny_scene)
    cam = tiny_cams[0]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    big = scenegen.look_camera(cam.pos, 0.0, 0.0, vy.NOALLOC_MAX_WIDTH + 16, 64)
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_render_noalloc(sc, cut, big)
    assert e.value.code == vy.VY_ERR_ARG
    torch.cuda.synchronize()
