"""Oracle: per-pixel front-to-back alpha blending (FP64). Test infrastructure only.

Section 3.1 "Rasterization" and Section 4.2 (Eq. 3): for a pixel, every
projected Gaussian i is visited in depth order (nearest first); its
transmittance is alpha_i = min(0.99, theta_i e^rho_i) with the power decay
rho_i = -1/2 d^T conic_i d at the pixel (d = pixel centre - mean2D); a Gaussian
with alpha_i < alpha* does not take part in the blend, the others contribute
alpha_i T c_i and multiply T by (1 - alpha_i).

Readings where the paper is silent: alpha* = 1/255 (the paper's effective rho
range [-5.55, 0] ends at ln(1/255)); blending stops, without blending the
Gaussian, once T (1 - alpha_i) would fall below 1e-4; rho is clamped to <= 0;
equal depths are ordered by node id; background black unless given; pixel
(i, j) is sampled at its centre (i + 0.5, j + 0.5). No tiles, no preemptive
filter and no LUT: every valid Gaussian is a candidate, pruned only by the
exact radius bound of oracle.project (plus 2 px slack, which cannot change the
result because the pruned alphas are below alpha* there).

LUT variant (Section 4.2, Eq. 5; used only when lut_m > 0): e^rho is replaced
by a table of the effective range [-5.55, 0] split into m intervals, read at
index round(rho / -5.55 * m). Readings: the table holds the m + 1 node values
e^(-5.55 k / m), k = 0..m (rounding to the nearest index can give 0..m, one
more than m entries), each rounded once to float32 as a device table stores
them; an index above m (rho below -5.55) reads node m, where theta e^rho is
below alpha* for theta <= 1.

Ambiguity accounting (for comparison with a float32 renderer): a pixel is
flagged when a decision that float32 rounding could flip is within a margin:
|ln alpha - ln alpha*| <= amb_alpha for a Gaussian visited up to termination,
|T(1 - alpha) - 1e-4| <= amb_t * 1e-4 at a blend, two consecutive contributors
with depths within amb_depth (relative), or a contributor within 1e-6
(relative) of the near plane; with the LUT also a Gaussian whose table
position -rho m / 5.55 lies within float32 reach of a rounding midpoint
(k + 1/2), the reach growing with the condition number of its conic.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
SLACK = 2.0


LUT_RANGE = 5.55


def lut_table(m):
    """The m + 1 node values e^(-5.55 k / m), k = 0..m (Section 4.2), as float32
    values (returned as float64)."""
    k = np.arange(m + 1, dtype=np.float64)
    return np.exp(-LUT_RANGE * k / m).astype(np.float32).astype(np.float64)


def lut_index(rho, m):
    """Eq. 5: round(rho / -5.55 * m), to the nearest integer (ties to even), at most m."""
    return np.minimum(np.rint(np.asarray(rho, np.float64) / -LUT_RANGE * m), m).astype(np.int64)


def lut_exp(rho, m):
    """e^rho read from the table (Section 4.2)."""
    return lut_table(m)[lut_index(rho, m)]


def conic_condition(conic):
    """lambda_max / lambda_min of the symmetric 2x2 conics [a, b, c] (n, 3)."""
    a, b, c = conic[:, 0], conic[:, 1], conic[:, 2]
    mid = 0.5 * (a + c)
    rad = np.sqrt(np.maximum(0.0, 0.25 * (a - c) ** 2 + b * b))
    return (mid + rad) / np.maximum(mid - rad, 1e-300)


def depth_order(proj):
    """Indices of valid Gaussians sorted by (depth, node id)."""
    v = np.nonzero(proj["valid"])[0]
    o = np.lexsort((proj["ids"][v], proj["depth"][v]))
    return v[o]


def render_pixels(proj, px, py, bg=(0.0, 0.0, 0.0), order=None, amb_alpha=2e-4, amb_t=2e-4, amb_depth=1e-6,
                  chunk=2048, lut_m=0, amb_lut=4e-6, signature=False):
    """Blend pixels with integer coordinates (px, py) (1-D arrays); lut_m > 0
    reads e^rho from the table of Section 4.2 with m = lut_m.

    Returns dict(rgb (P, 3), T (P,), n_contrib (P,), ambiguous (P,) bool), and
    with `signature` a per-pixel uint64 digest of which Gaussians it blended
    (equal digests: the same blend decisions)."""
    if order is None:
        order = depth_order(proj)
    px = np.asarray(px, np.int64)
    py = np.asarray(py, np.int64)
    P = len(px)
    cxp = px + 0.5
    cyp = py + 0.5
    m = proj["mean2d"][order]
    r = proj["radius"][order] + SLACK
    # candidates: squares intersecting the pixels' bounding box
    if P:
        x0, x1, y0, y1 = cxp.min(), cxp.max(), cyp.min(), cyp.max()
        keep = (m[:, 0] + r >= x0) & (m[:, 0] - r <= x1) & (m[:, 1] + r >= y0) & (m[:, 1] - r <= y1)
    else:
        keep = np.zeros(len(order), bool)
    cand = order[keep]
    mc, rc = m[keep], r[keep]
    con = proj["conic"][cand]
    th = proj["theta"][cand]
    rgb_g = proj["rgb"][cand]
    dep = proj["depth"][cand]
    nearm = proj["near_margin"][cand]
    if lut_m:
        table = lut_table(lut_m)
        lut_reach = amb_lut * (1.0 + conic_condition(con))   # float32 reach of -rho m / 5.55, relative
    T = np.ones(P)
    C = np.zeros((P, 3))
    done = np.zeros(P, bool)
    ncon = np.zeros(P, np.int64)
    amb = np.zeros(P, bool)
    sig = np.zeros(P, np.uint64)
    if signature:
        z = proj["ids"][cand].astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(1)
        z = (z ^ (z >> np.uint64(31))) * np.uint64(0xBF58476D1CE4E5B9)
        hv = z ^ (z >> np.uint64(29))
    prev_depth = np.full(P, np.nan)
    ln_amin = math.log(ALPHA_MIN)
    for s in range(0, len(cand), chunk):
        e = min(len(cand), s + chunk)
        dx = cxp[:, None] - mc[None, s:e, 0]
        dy = cyp[:, None] - mc[None, s:e, 1]
        inside = (np.abs(dx) <= rc[None, s:e]) & (np.abs(dy) <= rc[None, s:e])
        Q = con[None, s:e, 0] * dx * dx + 2.0 * con[None, s:e, 1] * dx * dy + con[None, s:e, 2] * dy * dy
        rho = np.minimum(0.0, -0.5 * Q)
        if lut_m:
            tpos = rho / -LUT_RANGE * lut_m
            ex = table[np.minimum(np.rint(tpos), lut_m).astype(np.int64)]
        else:
            ex = np.exp(rho)
        alpha = np.minimum(ALPHA_MAX, th[None, s:e] * ex)
        alpha = np.where(inside, alpha, 0.0)
        use = inside & (alpha >= ALPHA_MIN) & ~done[:, None]
        a = np.where(use, alpha, 0.0)
        Tafter = T[:, None] * np.cumprod(1.0 - a, axis=1)
        Tbefore = np.concatenate([T[:, None], Tafter[:, :-1]], axis=1)
        stop = Tafter < T_MIN                       # monotone along the row
        first_stop = stop & ~np.concatenate([np.zeros((P, 1), bool), stop[:, :-1]], axis=1)
        active = use & ~stop                        # blended
        w = np.where(active, a * Tbefore, 0.0)
        C += np.einsum("pk,kc->pc", w, rgb_g[s:e])   # einsum's own loops, not BLAS (threads)
        ncon += active.sum(axis=1)
        if signature:
            sig += np.where(active, hv[None, s:e], np.uint64(0)).sum(axis=1, dtype=np.uint64)
        relevant = (~stop | first_stop) & inside & ~done[:, None]
        with np.errstate(divide="ignore"):
            la = np.log(np.where(alpha > 0, alpha, 1e-300))
        amb |= np.any(relevant & (np.abs(la - ln_amin) <= amb_alpha), axis=1)
        amb |= np.any(use & relevant & (np.abs(Tafter - T_MIN) <= amb_t * T_MIN), axis=1)
        amb |= np.any(active & (nearm[None, s:e] <= 1e-6), axis=1)
        if lut_m:
            mid = np.abs(tpos - np.floor(tpos) - 0.5)
            amb |= np.any(relevant & (tpos < lut_m + 0.5) & (mid <= lut_reach[None, s:e] * (1.0 + tpos)), axis=1)
        # depth ties between consecutive contributors
        idx = np.where(active, np.arange(e - s)[None, :], -1)
        last = np.maximum.accumulate(idx, axis=1)
        prev_idx = np.concatenate([np.full((P, 1), -1), last[:, :-1]], axis=1)
        d_here = dep[None, s:e]
        d_prev = np.where(prev_idx >= 0, dep[s:e][np.maximum(prev_idx, 0)], prev_depth[:, None])
        tie = active & np.isfinite(d_prev) & (np.abs(d_here - d_prev) <= amb_depth * np.abs(d_here))
        amb |= np.any(tie, axis=1)
        has = last[:, -1] >= 0
        prev_depth = np.where(has, dep[s:e][np.maximum(last[:, -1], 0)], prev_depth)
        # carry state
        any_stop = stop.any(axis=1)
        T = np.where(any_stop, np.where(first_stop, Tbefore, 0.0).sum(axis=1), Tafter[:, -1])
        done |= any_stop
    bgv = np.asarray(bg, np.float64)
    out = dict(rgb=C + T[:, None] * bgv[None, :], T=T, n_contrib=ncon, ambiguous=amb)
    if signature:
        out["signature"] = sig
    return out


def render_image(proj, width, height, bg=(0.0, 0.0, 0.0), tiles=None, tile=16, threads=1, **kw):
    """Whole image (3, H, W) (or only the given tile indices, others NaN), plus
    T_final, n_contrib and the ambiguity mask (H, W). `threads` > 1 renders
    the tiles on that many threads (each tile's pixels as render_pixels
    computes them; only the work is split)."""
    order = depth_order(proj)
    img = np.full((3, height, width), np.nan)
    Tf = np.full((height, width), np.nan)
    nc = np.full((height, width), -1, np.int64)
    amb = np.zeros((height, width), bool)
    sig = np.zeros((height, width), np.uint64) if kw.get("signature") else None
    tx_n = (width + tile - 1) // tile
    ty_n = (height + tile - 1) // tile
    all_tiles = list(range(tx_n * ty_n) if tiles is None else tiles)

    def one(t):
        ty, tx = divmod(int(t), tx_n)
        xs = np.arange(tx * tile, min(width, (tx + 1) * tile))
        ys = np.arange(ty * tile, min(height, (ty + 1) * tile))
        PX, PY = np.meshgrid(xs, ys)
        return PX, PY, render_pixels(proj, PX.ravel(), PY.ravel(), bg=bg, order=order, **kw)

    if threads > 1 and len(all_tiles) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            results = list(ex.map(one, all_tiles))
    else:
        results = map(one, all_tiles)
    for PX, PY, r in results:
        img[:, PY.ravel(), PX.ravel()] = r["rgb"].T
        Tf[PY.ravel(), PX.ravel()] = r["T"]
        nc[PY.ravel(), PX.ravel()] = r["n_contrib"]
        amb[PY.ravel(), PX.ravel()] = r["ambiguous"]
        if sig is not None:
            sig[PY.ravel(), PX.ravel()] = r["signature"]
    out = dict(image=img, T=Tf, n_contrib=nc, ambiguous=amb)
    if sig is not None:
        out["signature"] = sig
    return out


def render_pixel_loop(proj, px: int, py: int, bg=(0.0, 0.0, 0.0), lut_m=0):
    """The definition as a plain loop over every valid Gaussian (one pixel,
    no pruning). Slow; used to pin render_pixels on tiny inputs."""
    order = depth_order(proj)
    table = lut_table(lut_m) if lut_m else None
    T = 1.0
    C = np.zeros(3)
    n = 0
    for i in order.tolist():
        dx = px + 0.5 - proj["mean2d"][i, 0]
        dy = py + 0.5 - proj["mean2d"][i, 1]
        A, B, Cc = proj["conic"][i]
        rho = min(0.0, -0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy))
        if lut_m:
            k = min(int(round(rho / -LUT_RANGE * lut_m)), lut_m)   # Python's round: ties to even
            ex = table[k]
        else:
            ex = math.exp(rho)
        alpha = min(ALPHA_MAX, proj["theta"][i] * ex)
        if alpha < ALPHA_MIN:
            continue
        t_next = T * (1.0 - alpha)
        if t_next < T_MIN:
            break
        C += alpha * T * proj["rgb"][i]
        T = t_next
        n += 1
    return C + T * np.asarray(bg, np.float64), T, n
