"""GPU checks on the plain renderer's workload: 2e6 leaves (about 4e6 nodes),
1280x720, the 120-frame walkthrough at tau = 2. Two sampled frames (the first
and a late one) against the FP64 oracle: the cut against the brute force over
every node, and tiles of the image, the two with the longest tile lists among
them; along the whole path, the temporal cut equals the full cut and the
alpha-filtered image equals the unfiltered one, bit for bit."""
import numpy as np
import pytest

import scenegen
from oracle import lod as olod, project as oproj, render as orender

from gpu_util import image_parity, require_gpu

pytestmark = pytest.mark.gpu

TAU = 2.0
THREADS = 16


@pytest.fixture(scope="module")
def med():
    vy = require_gpu()
    import torch
    cfg = scenegen.CONFIGS["med"]
    print(f"generating the {cfg.n_leaf}-leaf city", flush=True)
    host = scenegen.make_city(cfg)
    scene = vy.Scene(host)
    assert scene.validate() == 0
    cams = scenegen.walkthrough(cfg)
    assert len(cams) == 120
    ctx = vy.RenderContext(scene.n, cfg.width, cfg.height, 32 << 20)
    return vy, torch, cfg, host, scene, cams, ctx


@pytest.mark.parametrize("frame", [0, 110])
def test_cut_and_tiles_match_oracle(med, frame):
    vy, torch, cfg, host, scene, cams, ctx = med
    W, H = cfg.width, cfg.height
    cam = cams[frame]
    cut = vy.vy_lod_cut(scene, cam, TAU)
    F, C = cut.ids()
    res = olod.compare_cut(host, cam, TAU, F, C, threads=THREADS)
    print(f"frame {frame}: |F| {len(F)} |C| {len(C)}; cut {res}", flush=True)
    assert res["ok"], res
    img = vy.vy_render(scene, cut, cam, ctx).cpu().numpy()      # the plain renderer: unfiltered
    keys, vals, ranges = ctx.pairs(W, H)
    length = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    heavy = [int(t) for t in np.argsort(-length)[:2]]
    rng = np.random.default_rng(frame)
    tiles = sorted(set(heavy) | {int(t) for t in rng.choice(len(ranges), size=6, replace=False)})
    ref = orender.render_image(oproj.project_threaded(host, C, cam, threads=THREADS), W, H, tiles=tiles,
                               threads=THREADS)
    r = image_parity(img, ref)
    print(f"tiles {tiles} (pairs {[int(length[t]) for t in tiles]}): {r}", flush=True)
    assert r["ok"], r


def test_temporal_equals_full_and_filter_is_lossless_every_frame(med):
    vy, torch, cfg, host, scene, cams, ctx = med
    W, H = cfg.width, cfg.height
    state, whole = vy.Cut(scene), vy.Cut(scene)
    a = torch.empty((3, H, W), device="cuda")
    b = torch.empty_like(a)
    for i, cam in enumerate(cams):
        vy.vy_lod_cut(scene, cam, TAU, prev=state if i else None, out=state)
        vy.vy_lod_cut(scene, cam, TAU, out=whole)
        Ft, Ct = state.ids()
        Ff, Cf = whole.ids()
        assert np.array_equal(Ft, Ff) and np.array_equal(Ct, Cf), i
        vy.vy_render(scene, state, cam, ctx, image=a, alpha_filter=True)
        vy.check(ctx.status()[0])
        vy.vy_render(scene, whole, cam, ctx, image=b, alpha_filter=False)
        vy.check(ctx.status()[0])
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), i
