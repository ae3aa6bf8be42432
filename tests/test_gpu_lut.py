"""GPU checks of the LUT exponential of Section 4.2 (Eq. 5), through the C
ABI: with the table, filtered and unfiltered images stay bitwise equal and so
do the three walks; the image matches the oracle's LUT image (max abs 2e-3
over pixels whose table indices float32 rounding cannot flip, mean abs 1e-3
over all pixels, since a flipped index moves alpha by a factor e^(5.55/m));
it approaches the exact image as m grows."""
import numpy as np
import pytest

from oracle import project as oproj, render as orender
from paper_2506_02774_amd import quality

from gpu_util import image_parity, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny(tiny_scene):
    vy = require_gpu()
    sc = vy.Scene(tiny_scene)
    ctx = vy.RenderContext(sc.n, 256, 256, 1 << 22)
    return vy, sc, tiny_scene, ctx


def _img(vy, sc, cut, cam, ctx, **kw):
    out = vy.vy_render(sc, cut, cam, ctx, **kw).cpu().numpy()
    vy.check(ctx.status()[0])
    return out


@pytest.mark.parametrize("m", [8, 32, 128])
def test_lut_images(tiny, tiny_cams, m):
    vy, sc, host, ctx = tiny
    state = None
    for i, cam in enumerate(tiny_cams):
        state = vy.vy_lod_cut(sc, cam, 2.0, prev=state, out=state) if state is not None else vy.vy_lod_cut(sc, cam, 2.0)
        exact = _img(vy, sc, state, cam, ctx, alpha_filter=True)
        ref = None
        for filt in (False, True):
            for walk in (0, 1, 2):
                img = _img(vy, sc, state, cam, ctx, alpha_filter=filt, walk=walk, lut_entries=m)
                if ref is None:
                    ref = img
                assert np.array_equal(img.view(np.uint32), ref.view(np.uint32)), (i, filt, walk)
        if i % 3 == 0:
            F, C = state.ids()
            o = orender.render_image(oproj.project(host, C, cam), cam.width, cam.height, lut_m=m)
            r = image_parity(ref, o, max_abs=2e-3, mean_abs=1e-3)
            print(f"m={m} frame {i}: {r}; PSNR vs exact {quality.psnr(ref, exact):.2f} dB, "
                  f"SSIM {quality.ssim(ref, exact):.5f}", flush=True)
            assert r["ok"], r
            assert r["ambiguous"] <= 0.05 * r["n_pix"], r


def test_lut_approaches_exact(tiny, tiny_cams):
    vy, sc, host, ctx = tiny
    cam = tiny_cams[4]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    exact = _img(vy, sc, cut, cam, ctx, alpha_filter=True)
    p = [quality.psnr(_img(vy, sc, cut, cam, ctx, alpha_filter=True, lut_entries=m), exact) for m in (4, 16, 64)]
    print("PSNR m=4,16,64:", p, flush=True)
    assert p[0] < p[1] < p[2] and p[2] > 30.0


def test_lut_argument_errors(tiny, tiny_cams):
    vy, sc, host, ctx = tiny
    cam = tiny_cams[0]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    for bad in (dict(lut_entries=129), dict(lut_entries=-1), dict(lut_entries=16, split_min_pairs=64)):
        with pytest.raises(vy.VoyagerError) as e:
            vy.vy_render(sc, cut, cam, ctx, **bad)
        assert e.value.code == vy.VY_ERR_ARG
