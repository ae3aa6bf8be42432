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


EPS = 2.0 ** -24     # float32 unit roundoff
# Bounds on |GPU - FP64 oracle| for each projected attribute, in units of EPS
# times a per-Gaussian scale that follows the float32 operations (Section 3.1
# "Culling & Projection"; the scales are derived in the design notes):
K_MEAN, K_DEPTH, K_CONIC, K_RGB, K_THETA = 16.0, 8.0, 32.0, 64.0, 8.0


def projection_errors(vy, ctx, host, C, cam):
    """Per-attribute max of |GPU - oracle| / bound over the Gaussians both
    sides keep; all must be <= 1. Returns (ratios, n compared, n clamped)."""
    from oracle import sh as osh
    r0, r1, r2, br = ctx.projected(len(C))
    lo, hi = br[:, 0], br[:, 1]
    p = oproj.project(host, C, cam)
    gv = (lo != 0) | (hi != 0) | (r1[:, 3] > 0)
    # culling agrees except at the near plane / off-screen rect boundary
    assert np.all(p["valid"][gv] | (p["near_margin"][gv] < 1e-5))
    both = gv & p["valid"]
    f = float(np.float32(cam.fx))
    d = host.mean[C].astype(np.float64) - cam.pos.astype(np.float64)
    D = np.linalg.norm(d, axis=1)
    z = p["depth"]
    u = (p["mean2d"][:, 0] - cam.cx) / f          # true x/z and y/z (mean2D is not clamped)
    v = (p["mean2d"][:, 1] - cam.cy) / f
    uc = np.clip(u, -1.3 * cam.cx / f, 1.3 * (cam.width - cam.cx) / f)
    vc = np.clip(v, -1.3 * cam.cy / f, 1.3 * (cam.height - cam.cy) / f)
    clamped = both & ((uc != u) | (vc != v))
    out = {}
    # mean2D = f x/z + c: x, z carry ~EPS |mu - cam| each
    bm = EPS * (f * D * (1 + np.abs(u) + np.abs(v)) / z + np.abs(p["mean2d"]).max(axis=1))
    out["mean2d"] = np.max(np.abs(r0[:, :2] - p["mean2d"]).max(axis=1)[both] / (K_MEAN * bm[both]))
    out["depth"] = np.max(np.abs(r1[both, 3] - z[both]) / (K_DEPTH * EPS * D[both]))
    # conic (stored as rho coefficients -a/2, -b, -c/2): norm-wise, times the
    # condition number of Sigma2 (the inverse) and the Jacobian's growth
    ref = np.stack([-0.5 * p["conic"][:, 0], -p["conic"][:, 1], -0.5 * p["conic"][:, 2]], 1)
    got = np.stack([r0[:, 2], r0[:, 3], r1[:, 0]], 1)
    cov = p["cov2d"]
    mid = 0.5 * (cov[:, 0] + cov[:, 2])
    rad = np.sqrt(0.25 * (cov[:, 0] - cov[:, 2]) ** 2 + cov[:, 1] ** 2)
    cond = (mid + rad) / (mid - rad)
    bc = EPS * cond * (D / z) * (1 + np.abs(uc) + np.abs(vc)) ** 2 * np.abs(ref).max(axis=1)
    out["conic"] = np.max(np.abs(got - ref).max(axis=1)[both] / (K_CONIC * bc[both]))
    # SH colour: a sum of 16 terms per channel (the [0, 1] clamp only shrinks errors)
    Y = osh.basis(d / D[:, None])
    mag = np.einsum("nk,nkc->nc", np.abs(Y), np.abs(host.sh[C].astype(np.float64)))
    out["rgb"] = np.max((np.abs(r2[:, :3] - p["rgb"]) / (K_RGB * EPS * (1 + mag)))[both])
    out["theta"] = np.max(np.abs(r1[both, 1] - p["theta"][both]) / (K_THETA * EPS * p["theta"][both]))
    # per-axis pixel extents ceil(3.33 sqrt(Sigma2_xx)), ceil(3.33 sqrt(Sigma2_yy)) (1 px ceil flips allowed)
    e = r2[both, 3].view(np.uint32)
    rx, ry = (e & 0xFFFF).astype(float), (e >> 16).astype(float)
    assert np.all(np.abs(rx - np.ceil(3.33 * np.sqrt(cov[both, 0]))) <= 1)
    assert np.all(np.abs(ry - np.ceil(3.33 * np.sqrt(cov[both, 2]))) <= 1)
    # the box is inside the oracle's square bound
    assert np.all(rx <= p["radius"][both] + 1) and np.all(ry <= p["radius"][both] + 1)
    return out, int(both.sum()), int(clamped.sum())


def test_projection_matches_oracle(frame):
    vy, sc, host, ctx, cam, cut, C = frame
    vy.vy_render(sc, cut, cam, ctx)
    ratios, n, nclamp = projection_errors(vy, ctx, host, C, cam)
    print(f"{n} Gaussians ({nclamp} under the Jacobian clamp); error / bound: "
          + ", ".join(f"{k} {v:.3f}" for k, v in ratios.items()), flush=True)
    assert n > 0.5 * len(C)
    assert all(v <= 1.0 for v in ratios.values()), ratios


def test_projection_under_the_jacobian_clamp():
    """Gaussians whose centre lies past 1.3x the half-extent of the image in
    x/z or y/z (the Jacobian takes the clamped ratio) but whose footprint
    still reaches the image: projected as the oracle projects them."""
    vy = require_gpu()
    W, H = 192, 128
    rng = np.random.default_rng(21)
    n = 3000
    z = rng.uniform(2.0, 12.0, n)
    su = rng.choice([-1.0, 1.0], n) * rng.uniform(0.8, 1.6, n)      # beyond +-1.3 tan 30 = +-0.75
    sv = rng.uniform(-1.2, 1.2, n)
    mean = np.stack([su * z, sv * z * H / W, z], 1).astype(np.float32)
    ls = rng.uniform(-0.7, 0.4, (n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    lg = rng.normal(0, 1.5, n).astype(np.float32)
    shc = rng.normal(0, 0.2, (n, 16, 3)).astype(np.float32)
    shc[:, 0] += 0.5
    host = scenegen.build_hierarchy(dict(mean=mean, log_scale=ls, quat=q, opacity_logit=lg, sh=shc))
    cam = scenegen.identity_camera(W, H)
    sc = vy.Scene(host)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 22)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    F, C = cut.ids()
    vy.vy_render(sc, cut, cam, ctx)
    ratios, nb, nclamp = projection_errors(vy, ctx, host, C, cam)
    print(f"{nb} Gaussians ({nclamp} under the Jacobian clamp); error / bound: "
          + ", ".join(f"{k} {v:.3f}" for k, v in ratios.items()), flush=True)
    assert nclamp > 200
    assert all(v <= 1.0 for v in ratios.values()), ratios


@pytest.mark.parametrize("filt", [False, True])
def test_sorted_pairs(frame, filt):
    vy, sc, host, ctx, cam, cut, C = frame
    vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt)
    keys, vals, ranges = ctx.pairs(cam.width, cam.height)
    r0, r1, r2, br = ctx.projected(len(C))
    lo, hi, mask = br[:, 0], br[:, 1], br[:, 2]
    count = np.where(mask != 0, br[:, 3] & 0xFF, br[:, 3])   # small rects: the pixel box above the count
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
    lx, hx, mx = check_key_boxes(ctx, cam, keys, vals, r0, r2)
    # and it is not the whole tile for most pairs (the far city's Gaussians are small)
    assert ((hx - lx) < 15).mean() > 0.3, ((hx - lx) < 15).mean()


def check_key_boxes(ctx, cam, keys, vals, r0, r2):
    """Each key's pixel box (bits 16..31: first and last column, first and
    last row) holds every pixel of its tile where the blend's pixel rule,
    evaluated in float32 as the blend does, lets the Gaussian in. Returns the
    boxes' first and last columns and the pairs' centres' x."""
    tx_n = (cam.width + 15) // 16
    raw, _, _ = ctx.pairs(cam.width, cam.height, raw=True)
    assert np.array_equal(raw & 0xFFFF, keys)
    box = raw >> 16
    lx, hx, ly, hy = box & 15, (box >> 4) & 15, (box >> 8) & 15, (box >> 12) & 15
    tx, ty = (keys % tx_n).astype(np.int64), (keys // tx_n).astype(np.int64)
    ext = np.ascontiguousarray(r2[vals, 3]).view(np.uint32)
    rx, ry = (ext & 0xFFFF).astype(np.float32), (ext >> 16).astype(np.float32)
    mx, my = r0[vals, 0].astype(np.float32), r0[vals, 1].astype(np.float32)
    c = np.arange(16)
    cx = (tx[:, None] * 16 + c[None, :]).astype(np.float32) + np.float32(0.5)
    cy = (ty[:, None] * 16 + c[None, :]).astype(np.float32) + np.float32(0.5)
    okx = np.abs(mx[:, None] - cx) <= rx[:, None]
    oky = np.abs(my[:, None] - cy) <= ry[:, None]
    assert not (okx & ((c[None, :] < lx[:, None]) | (c[None, :] > hx[:, None]))).any()
    assert not (oky & ((c[None, :] < ly[:, None]) | (c[None, :] > hy[:, None]))).any()
    return lx, hx, mx


@pytest.mark.parametrize("filt", [False, True])
def test_key_boxes_far_centres(filt):
    """Key boxes of Gaussians centred far outside the image (up to about
    27 000 pixels to the side) whose long, thin footprints still reach into
    it: the rounding slack of the box grows with the centre's magnitude, and
    the boxes stay supersets of the pixel rule there too."""
    vy = require_gpu()
    W, H = 64, 48
    rng = np.random.default_rng(33)
    n = 4000
    z = rng.uniform(2.0, 12.0, n)
    u = rng.choice([-1.0, 1.0], n) * np.exp(rng.uniform(np.log(2.0), np.log(500.0), n))   # x / z
    v = rng.uniform(-0.4, 0.4, n)
    x = u * z
    mean = np.stack([x, v * z, z], 1).astype(np.float32)
    # axis-aligned, long in x (about a third of the distance to the image's
    # centre line, so that 3.33 sigma reaches back into the image or just
    # misses it) and thin in y and z
    ls = np.stack([np.log(np.abs(x) * rng.uniform(0.28, 0.4, n)),
                   rng.uniform(-3.0, -1.5, n), rng.uniform(-3.0, -1.5, n)], 1).astype(np.float32)
    q = np.tile(np.array([1.0, 0.0, 0.0, 0.0], np.float32), (n, 1))
    lg = rng.uniform(1.0, 4.0, n).astype(np.float32)
    shc = rng.normal(0, 0.2, (n, 16, 3)).astype(np.float32)
    shc[:, 0] += 0.5
    host = scenegen.build_hierarchy(dict(mean=mean, log_scale=ls, quat=q, opacity_logit=lg, sh=shc))
    cam = scenegen.identity_camera(W, H)
    sc = vy.Scene(host)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 22)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    F, C = cut.ids()
    vy.vy_render(sc, cut, cam, ctx, alpha_filter=filt)
    vy.check(ctx.status()[0])
    keys, vals, ranges = ctx.pairs(W, H)
    r0, r1, r2, br = ctx.projected(len(C))
    lx, hx, mx = check_key_boxes(ctx, cam, keys, vals, r0, r2)
    far = np.abs(mx) > 5000.0
    print(f"{len(keys)} pairs, {int(far.sum())} of centres beyond 5000 px (max {np.abs(mx).max():.0f})", flush=True)
    assert far.sum() > 50
