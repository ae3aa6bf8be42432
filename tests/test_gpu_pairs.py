"""GPU checks of the intermediate stages (through the C ABI): projected
attributes against the FP64 oracle projection, and the sorted pair list
against its definition: every (tile, Gaussian) pair of each Gaussian's tile
rect exactly once, ordered by (tile, depth, node id)."""
import numpy as np
import pytest

import scenegen
from oracle import project as oproj

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frame(tiny_scene, tiny_cams):
    vy = require_gpu()
    sc = vy.Scene(tiny_scene)
    ctx = vy.RenderContext(sc.n, 256, 256, 1 << 22)
    cam = tiny_cams[4]
    cut = vy.vy_lod_cut(sc, cam, 2.0)
    F, C = cut.ids()
    return vy, sc, tiny_scene, ctx, cam, cut, C


def test_projection_matches_oracle(frame):
    vy, sc, host, ctx, cam, cut, C = frame
    vy.vy_render(sc, cut, cam, ctx)
    r0, r1, r2, br = ctx.projected(len(C))
    lo, hi = br[:, 0], br[:, 1]
    p = oproj.project(host, C, cam)
    gv = (lo != 0) | (hi != 0) | (r1[:, 3] > 0)
    both = gv & p["valid"]
    assert both.sum() > 0.5 * len(C)
    # culling agrees except at the near plane / off-screen rect boundary
    assert np.all(p["valid"][gv] | (p["near_margin"][gv] < 1e-5))
    np.testing.assert_allclose(r0[both, 0], p["mean2d"][both, 0], atol=2e-3, rtol=1e-5)
    np.testing.assert_allclose(r0[both, 1], p["mean2d"][both, 1], atol=2e-3, rtol=1e-5)
    np.testing.assert_allclose(r1[both, 3], p["depth"][both], rtol=1e-6)
    np.testing.assert_allclose(r1[both, 1], p["theta"][both], rtol=1e-6)
    np.testing.assert_allclose(r2[both, :3], p["rgb"][both], atol=2e-6)
    # rho coefficients (A, B, C) = (-a/2, -b, -c/2), relative to the conic's scale
    ref = np.stack([-0.5 * p["conic"][:, 0], -p["conic"][:, 1], -0.5 * p["conic"][:, 2]], 1)[both]
    got = np.stack([r0[both, 2], r0[both, 3], r1[both, 0]], 1)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.max(np.abs(got - ref) / scale) < 1e-3
    # per-axis pixel extents ceil(3.33 sqrt(Sigma2_xx)), ceil(3.33 sqrt(Sigma2_yy)) (1 px ceil flips allowed)
    e = r2[both, 3].view(np.uint32)
    rx, ry = (e & 0xFFFF).astype(float), (e >> 16).astype(float)
    assert np.all(np.abs(rx - np.ceil(3.33 * np.sqrt(p["cov2d"][both, 0]))) <= 1)
    assert np.all(np.abs(ry - np.ceil(3.33 * np.sqrt(p["cov2d"][both, 2]))) <= 1)
    # the box is inside the oracle's square bound
    assert np.all(rx <= p["radius"][both] + 1) and np.all(ry <= p["radius"][both] + 1)


@pytest.mark.parametrize("filt", [False, True])
def test_sorted_pairs(frame, filt):
    vy, sc, host, ctx, cam, cut, C = frame
    vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt)
    keys, vals, ranges = ctx.pairs(cam.width, cam.height)
    r0, r1, r2, br = ctx.projected(len(C))
    lo, hi, mask, count = br[:, 0], br[:, 1], br[:, 2], br[:, 3]
    tx_n = (cam.width + 15) // 16
    # ranges partition the pair list by tile, in tile order
    nz = ranges[:, 1] > ranges[:, 0]
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    for t in np.nonzero(nz)[0]:
        a, b = ranges[t]
        assert np.all(keys[a:b] == t)
    assert (ranges[:, 1] - ranges[:, 0]).sum() == len(keys)
    # within a tile: strictly increasing (depth, cut position)
    d = r1[vals, 3]
    same = keys[1:] == keys[:-1]
    inc = (d[1:] > d[:-1]) | ((d[1:] == d[:-1]) & (vals[1:] > vals[:-1]))
    assert np.all(inc[same])
    # the pair set: unfiltered = every tile of every rect; filtered = a subset
    got = set(zip(keys.tolist(), vals.tolist()))
    assert len(got) == len(keys)
    exp = set()
    for g in np.nonzero((lo != 0) | (hi != 0) | (r1[:, 3] > 0))[0]:
        x0, y0, x1, y1 = lo[g] & 0xFFFF, lo[g] >> 16, hi[g] & 0xFFFF, hi[g] >> 16
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                exp.add((ty * tx_n + tx, int(g)))
    if filt:
        assert got <= exp
    else:
        assert got == exp
    # pair counts: per Gaussian, as many pairs as its record says; for rects of
    # at most 32 tiles exactly the tiles of its kept-tile mask (row-major bits)
    per_g = np.bincount(vals, minlength=len(C))
    assert np.array_equal(per_g, count.astype(np.int64))
    w = (hi & 0xFFFF).astype(np.int64) - (lo & 0xFFFF) + 1
    h = (hi >> 16).astype(np.int64) - (lo >> 16) + 1
    small = (count > 0) & (w * h <= 32)
    assert small.sum() > 0 and np.all(mask[(count > 0) & ~small] == 0)
    bits = {}
    for t, g in got:
        if small[g]:
            x0, y0 = lo[g] & 0xFFFF, lo[g] >> 16
            k = (t // tx_n - y0) * w[g] + (t % tx_n - x0)
            bits[g] = bits.get(g, 0) | (1 << int(k))
    assert all(bits.get(int(g), 0) == int(mask[g]) for g in np.nonzero(small)[0])
