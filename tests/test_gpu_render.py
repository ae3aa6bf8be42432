"""GPU parity of splatting (through the C ABI): images against the FP64
oracle within max-abs 2e-3 (non-ambiguous pixels) and mean-abs 1e-4, and the
alpha-filtered image bitwise equal to the unfiltered one."""
import numpy as np
import pytest

import scenegen
from oracle import project as oproj, render as orender

from gpu_util import image_parity, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny(tiny_scene):
    vy = require_gpu()
    sc = vy.Scene(tiny_scene)
    ctx = vy.RenderContext(sc.n, 256, 256, 1 << 22)
    return vy, sc, tiny_scene, ctx


def _render_both(vy, sc, cut, cam, ctx, bg=(0.0, 0.0, 0.0)):
    a = vy.vy_render(sc, cut, cam, ctx, alpha_filter=False, bg=bg).cpu().numpy()
    rc, npairs_a, nvis_a = ctx.status()
    vy.check(rc)
    b = vy.vy_render(sc, cut, cam, ctx, alpha_filter=True, bg=bg).cpu().numpy()
    rc, npairs_b, nvis_b = ctx.status()
    vy.check(rc)
    return a, b, npairs_a, npairs_b


def test_walkthrough_images_match_oracle(tiny, tiny_cams):
    vy, sc, host, ctx = tiny
    state = None
    for i, cam in enumerate(tiny_cams):
        state = vy.vy_lod_cut(sc, cam, 2.0, prev=state, out=state) if state is not None else \
            vy.vy_lod_cut(sc, cam, 2.0)
        F, C = state.ids()
        a, b, pa, pb = _render_both(vy, sc, state, cam, ctx)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"frame {i}: filtered != unfiltered"
        assert pb <= pa
        ref = orender.render_image(oproj.project(host, C, cam), cam.width, cam.height)
        res = image_parity(a, ref)
        print(f"frame {i}: |C|={len(C)} pairs {pa} -> {pb} (filtered) {res}", flush=True)
        assert res["ok"], res


def test_random_gaussians_ragged_image():
    vy = require_gpu()
    W, H = 100, 37
    leaves = scenegen.random_gaussians(3000, 4, W, H, depth_range=(1.0, 40.0), scale_range=(-3.5, 0.5))
    L = dict(mean=leaves.mean, log_scale=leaves.log_scale, quat=leaves.quat,
             opacity_logit=leaves.opacity_logit, sh=leaves.sh)
    host = scenegen.build_hierarchy(L)
    sc = vy.Scene(host)
    cam = scenegen.identity_camera(W, H)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 22)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    F, C = cut.ids()
    assert np.all(host.child_count[C] == 0) and len(C) > 1000
    for bg in [(0.0, 0.0, 0.0), (0.25, 0.5, 1.0)]:
        a, b, pa, pb = _render_both(vy, sc, cut, cam, ctx, bg=bg)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        ref = orender.render_image(oproj.project(host, C, cam), W, H, bg=bg)
        res = image_parity(a, ref)
        print(bg, res, pa, pb, flush=True)
        assert res["ok"], res
        # both blend walks on wide anisotropic Gaussians, with and without the filter
        for filt in (False, True):
            imgs = [vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, bg=bg, walk=w).cpu().numpy()
                    for w in (1, 2)]
            assert np.array_equal(imgs[0].view(np.uint32), imgs[1].view(np.uint32))
            assert np.array_equal(imgs[0].view(np.uint32), a.view(np.uint32))


def test_empty_cut_gives_background(tiny):
    vy, sc, host, ctx = tiny
    cam = scenegen.look_camera([0.0, 0.0, 5000.0], 0.0, 1.2, 64, 48)
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    img = vy.vy_render(sc, cut, cam, ctx, bg=(0.1, 0.2, 0.3)).cpu().numpy()
    rc, npairs, nvis = ctx.status()
    vy.check(rc)
    assert npairs == 0 and nvis == 0
    assert np.all(img[0] == np.float32(0.1)) and np.all(img[2] == np.float32(0.3))


def test_tiny_images(tiny, tiny_cams):
    vy, sc, host, ctx = tiny
    cam0 = tiny_cams[2]
    for W, H in [(1, 1), (17, 3), (16, 16), (33, 250)]:
        cam = scenegen.look_camera(cam0.pos, 0.3, 0.0, W, H)
        cut = vy.vy_lod_cut(sc, cam, 2.0)
        F, C = cut.ids()
        a, b, pa, pb = _render_both(vy, sc, cut, cam, ctx)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        ref = orender.render_image(oproj.project(host, C, cam), W, H)
        res = image_parity(a, ref)
        assert res["ok"], (W, H, res)


def test_pair_overflow_reported(tiny, tiny_cams):
    vy, sc, host, _ = tiny
    ctx = vy.RenderContext(sc.n, 256, 256, 1000)
    cam = tiny_cams[0]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    vy.vy_render(sc, cut, cam, ctx)
    rc, need, nvis = ctx.status()
    assert rc == vy.VY_ERR_CAPACITY and need > 1000
    with pytest.raises(vy.VoyagerError):
        vy.vy_render(sc, cut, scenegen.identity_camera(512, 512), ctx)


@pytest.mark.parametrize("split_min", [1, 24, 300])
def test_split_blend_is_bitwise_identical(tiny, tiny_cams, split_min):
    """Tiles blended over several workgroups (depth-bin jobs + composite) give
    exactly the image, final transmittance and contributor counts of the
    one-piece blend, with and without the alpha filter."""
    vy, sc, host, ctx = tiny
    for cam in tiny_cams[::3]:
        cut = vy.vy_lod_cut(sc, cam, 2.0)
        ref = vy.vy_render(sc, cut, cam, ctx, split_min_pairs=1 << 30, save_state=True).cpu().numpy()
        T_ref, N_ref = ctx.saved(cam.width, cam.height)
        for filt in (False, True):
            img = vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, split_min_pairs=split_min,
                               save_state=True).cpu().numpy()
            rc, npairs, nvis = ctx.status()
            vy.check(rc)
            T, N = ctx.saved(cam.width, cam.height)
            assert np.array_equal(img.view(np.uint32), ref.view(np.uint32)), (split_min, filt)
            assert np.array_equal(T.view(np.uint32), T_ref.view(np.uint32))
            assert np.array_equal(N, N_ref)


def test_saved_state_matches_oracle(tiny, tiny_cams):
    vy, sc, host, ctx = tiny
    cam = tiny_cams[5]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    F, C = cut.ids()
    vy.vy_render(sc, cut, cam, ctx, save_state=True, split_min_pairs=64)
    T, N = ctx.saved(cam.width, cam.height)
    ref = orender.render_image(oproj.project(host, C, cam), cam.width, cam.height)
    ok = ~ref["ambiguous"]
    assert np.max(np.abs(T[ok] - ref["T"][ok])) < 2e-3
    assert np.mean(N[ok] == ref["n_contrib"][ok]) > 0.999


@pytest.mark.parametrize("filt", [False, True])
def test_saved_evaluation_counts(tiny, tiny_cams, filt):
    """Per-pixel evaluation counts of the one-piece blend: every pixel walks its
    tile's sorted list up to and including the entry that ends it (Section 3.1,
    early termination), so n_contrib <= n_eval <= the tile's list length, and a
    pixel whose list ran out evaluated all of it. Split jobs report -1."""
    vy, sc, host, ctx = tiny
    cam = tiny_cams[4]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, save_state=True)
    T, N, E = ctx.saved(cam.width, cam.height, evals=True)
    keys, vals, ranges = ctx.pairs(cam.width, cam.height)
    tx = (cam.width + 15) // 16
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    t = (ys // 16) * tx + xs // 16
    L = (ranges[:, 1].astype(np.int64) - ranges[:, 0].astype(np.int64))[t]
    assert (E >= N).all() and (E <= L).all()
    assert (E < L).any() and (E == L).any()
    vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, save_state=True, split_min_pairs=1)
    _, _, E2 = ctx.saved(cam.width, cam.height, evals=True)
    assert (E2 == -1).any()
    assert (E2[E2 >= 0] == E[E2 >= 0]).all()
    assert ((E2 == -1) | (E2 >= 0)).all()


@pytest.mark.parametrize("filt", [False, True])
def test_walks_are_bitwise_identical(tiny, tiny_cams, filt):
    """The band walk, the per-pixel walk and the automatic choice between them
    evaluate the same (Gaussian, pixel) pairs with the same arithmetic: images,
    final transmittance, contributor and evaluation counts agree bit for bit."""
    vy, sc, host, ctx = tiny
    for cam in tiny_cams[::2]:
        cut = vy.vy_lod_cut(sc, cam, 2.0)
        out = []
        for walk in (0, 1, 2):
            img = vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, save_state=True, walk=walk).cpu().numpy()
            vy.check(ctx.status()[0])
            T, N, E = ctx.saved(cam.width, cam.height, evals=True)
            out.append((img.view(np.uint32), T.view(np.uint32), N, E))
        for o in out[1:]:
            for a, b in zip(out[0], o):
                assert np.array_equal(a, b)
    with pytest.raises(vy.VoyagerError):
        vy.vy_render(sc, cut, tiny_cams[0], ctx, walk=3)
    with pytest.raises(vy.VoyagerError):
        vy.vy_render(sc, cut, tiny_cams[0], ctx, band_jobs=3)


@pytest.mark.parametrize("n,dim", [(60000, 0.0), (60000, 4.0), (130000, 0.0), (130000, 4.0), (130000, 8.0)])
def test_heavy_tiles_band_jobs(n, dim):
    """Tiles with more than 4096 pairs are blended band by band by separate
    waves in the automatic mode, as halves of bands (band_jobs 1, the default
    of vy_render) or whole bands (band_jobs 2); the image equals the workgroup
    walks bit for bit (with and without the filter) and matches the oracle.
    `dim` lowers the opacity logits so that pixels stop later or never."""
    vy = require_gpu()
    W, H = 64, 48
    leaves = scenegen.random_gaussians(n, 11, W, H, depth_range=(1.0, 60.0), scale_range=(-4.0, -1.0))
    L = dict(mean=leaves.mean, log_scale=leaves.log_scale, quat=leaves.quat,
             opacity_logit=(leaves.opacity_logit - np.float32(dim)).astype(np.float32), sh=leaves.sh)
    host = scenegen.build_hierarchy(L)
    sc = vy.Scene(host)
    cam = scenegen.identity_camera(W, H)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 22)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    F, C = cut.ids()
    imgs, longest = {}, {}
    for filt in (False, True):
        for walk in (0, 1, 2):
            imgs[filt, walk] = vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, walk=walk).cpu().numpy()
            vy.check(ctx.status()[0])
        for bj in (1, 2):
            imgs[filt, 0, bj] = vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt, band_jobs=bj).cpu().numpy()
        keys, vals, ranges = ctx.pairs(W, H)
        longest[filt] = int((ranges[:, 1] - ranges[:, 0]).max())
    assert longest[False] > (8192 if n > 100000 else 4096) and (dim > 0 or longest[True] > 4096), longest
    ref_img = imgs[False, 1].view(np.uint32)
    for k, v in imgs.items():
        assert np.array_equal(v.view(np.uint32), ref_img), k
    tiles = None if n < 100000 else [0, 5, 11]
    ref = orender.render_image(oproj.project(host, C, cam), W, H, tiles=tiles)
    res = image_parity(imgs[True, 0], ref)
    print(dim, res, flush=True)
    assert res["ok"], res


def test_measured_peaks_are_plausible():
    """The probe kernels behind the rooflines: FP32 FMA without packed
    instructions can reach at most half the chip's 157.3 TFLOP/s (packed)
    peak, and the exponential runs at a quarter of the FMA rate or less."""
    vy = require_gpu()
    p = vy.measure_peaks()
    print(p, flush=True)
    assert 10.0 < p["fma_fp32_tflops"] <= 0.5 * 157.3 * 1.05
    assert 50.0 < p["exp_f32_gops"] <= 1e3 * p["fma_fp32_tflops"] / 2
