"""GPU checks at the full city scale (18M leaves, 36M nodes, 1920x1080, tau =
2 px), with the contexts and options the benchmark times: one frame's cut
against the oracle's brute force over every node, and sampled tiles of its
image (the heaviest, horizon tiles among them) against the oracle; along a
stretch of the walkthrough, temporal == full cuts and filtered == unfiltered
images bit for bit at tau = 1, 2 and 4, and one more frame against the oracle
at tau = 1 and at tau = 4; the walkthrough renderer with four frames in flight (the
caller's stream as the first slot) equal to the frame loop, frame by frame."""
import numpy as np
import pytest

import scenegen
from oracle import lod as olod, project as oproj, render as orender

from gpu_util import image_parity, require_gpu

pytestmark = pytest.mark.gpu

TAU = 2.0
MAX_PAIRS = 96 << 20


@pytest.fixture(scope="module")
def full():
    vy = require_gpu()
    import torch
    cfg = scenegen.CONFIGS["full"]
    print(f"generating the {cfg.n_leaf}-leaf city", flush=True)
    host = scenegen.make_city(cfg)
    scene = vy.Scene(host)
    assert scene.validate() == 0
    cams = scenegen.walkthrough(cfg, frames=300)
    ctx = vy.RenderContext(scene.n, cfg.width, cfg.height, MAX_PAIRS)
    return vy, torch, cfg, host, scene, cams, ctx


def test_cut_and_sampled_tiles_match_oracle(full):
    vy, torch, cfg, host, scene, cams, ctx = full
    W, H = cfg.width, cfg.height
    cam = cams[150]
    cut = vy.vy_lod_cut(scene, cam, TAU)
    F, C = cut.ids()
    print(f"|F| {len(F)} |C| {len(C)}; oracle cut over {scene.n} nodes", flush=True)
    res = olod.compare_cut(host, cam, TAU, F, C)
    assert res["ok"], res
    img = vy.vy_render(scene, cut, cam, ctx, alpha_filter=True).cpu().numpy()
    keys, vals, ranges = ctx.pairs(W, H)
    length = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    heavy = [int(t) for t in np.argsort(-length)[:2]]          # the longest tile lists (the horizon)
    rng = np.random.default_rng(11)
    tiles = sorted(set(heavy) | {int(t) for t in rng.choice(len(ranges), size=6, replace=False)})
    print(f"oracle tiles {tiles} (pairs {[int(length[t]) for t in tiles]})", flush=True)
    ref = orender.render_image(oproj.project(host, C, cam), W, H, tiles=tiles)
    r = image_parity(img, ref)
    assert r["ok"], r


@pytest.mark.parametrize("tau,frame", [(1.0, 60), (4.0, 240)])
def test_other_taus_match_oracle(full, tau, frame):
    """tau = 1 (the heaviest cut) and tau = 4: the cut against the brute force
    and sampled tiles, the heaviest among them, against the oracle."""
    vy, torch, cfg, host, scene, cams, ctx = full
    W, H = cfg.width, cfg.height
    cam = cams[frame]
    cut = vy.vy_lod_cut(scene, cam, tau)
    F, C = cut.ids()
    res = olod.compare_cut(host, cam, tau, F, C, threads=16)
    print(f"tau {tau} frame {frame}: |F| {len(F)} |C| {len(C)}; cut {res}", flush=True)
    assert res["ok"], res
    img = vy.vy_render(scene, cut, cam, ctx, alpha_filter=True).cpu().numpy()
    vy.check(ctx.status()[0])
    keys, vals, ranges = ctx.pairs(W, H)
    length = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    heavy = [int(t) for t in np.argsort(-length)[:2]]
    rng = np.random.default_rng(frame)
    tiles = sorted(set(heavy) | {int(t) for t in rng.choice(len(ranges), size=4, replace=False)})
    ref = orender.render_image(oproj.project_threaded(host, C, cam, threads=16), W, H, tiles=tiles, threads=16)
    r = image_parity(img, ref)
    print(f"tiles {tiles} (pairs {[int(length[t]) for t in tiles]}): {r}", flush=True)
    assert r["ok"], r


@pytest.mark.parametrize("tau", [1.0, 2.0, 4.0])
def test_temporal_equals_full_and_filter_is_lossless(full, tau):
    vy, torch, cfg, host, scene, cams, ctx = full
    W, H = cfg.width, cfg.height
    state, whole = vy.Cut(scene), vy.Cut(scene)
    a = torch.empty((3, H, W), device="cuda")
    b = torch.empty_like(a)
    for i in range(0, 40, 4):      # every fourth frame: larger steps between the temporal searches
        cam = cams[i]
        vy.vy_lod_cut(scene, cam, tau, prev=state if i else None, out=state)
        vy.vy_lod_cut(scene, cam, tau, out=whole)
        Ft, Ct = state.ids()
        Ff, Cf = whole.ids()
        assert np.array_equal(Ft, Ff) and np.array_equal(Ct, Cf), i
        vy.vy_render(scene, state, cam, ctx, image=a, alpha_filter=True)
        vy.check(ctx.status()[0])
        vy.vy_render(scene, whole, cam, ctx, image=b, alpha_filter=False)
        vy.check(ctx.status()[0])
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), i


def test_four_frames_in_flight_equal_frame_loop(full):
    vy, torch, cfg, host, scene, cams, ctx = full
    from paper_2506_02774_amd.serving import STATS_DTYPE
    W, H = cfg.width, cfg.height
    path = cams[100:112]
    cut = vy.Cut(scene)
    ref = []
    for i, cam in enumerate(path):
        vy.vy_lod_cut(scene, cam, TAU, prev=cut if i else None, out=cut)
        ref.append(vy.vy_render(scene, cut, cam, ctx, alpha_filter=True))
    depth = 4
    cuts = [vy.Cut(scene) for _ in range(depth)]
    ctxs = [vy.RenderContext(scene.n, W, H, MAX_PAIRS) for _ in range(depth)]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(depth - 1)]
    images = [torch.empty((3, H, W), device="cuda") for _ in path]
    stats = torch.zeros((len(path), 4), dtype=torch.int64, device="cuda")
    vy.vy_walkthrough(scene, path, TAU, cuts, ctxs, images, streams=streams, alpha_filter=True, stats=stats)
    torch.cuda.synchronize()
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
    assert not st["flags"].any()
    for i in range(len(path)):
        assert torch.equal(images[i].view(torch.int32), ref[i].view(torch.int32)), i
