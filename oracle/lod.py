"""Oracle: the LoD cut by brute force (FP64). Test infrastructure only.

Follows Section 3.1 "Cut Finding": walking the LoD tree top-down, a node is
selected when the projected dimension of its Gaussian is below the LoD
granularity tau while its parent's is above. The paper does not define the
projected dimension or say how nodes outside the view frustum are handled
(Section 3.1 "LoD Tree" says the tree also identifies the Gaussians inside the
frustum). The readings used here:

* vis(n):  the node's AABB is not entirely outside any of the five frustum
           half-spaces (4 side planes through the camera centre, near plane),
           tested with the "positive vertex" of the box;
* ext(n):  the longest side of the node's AABB;
* dist(n): Euclidean distance from the camera centre to the AABB (0 inside);
* expand(n) <=> n has children AND vis(n) AND f * ext(n) > tau * dist(n)
           (f = fx; strict ">", so a tie at tau does not expand);
* frontier F = { n : not expand(n) and (n is the root or expand(parent(n))) };
* cut      C = F intersected with vis.

Because AABB(child) is contained in AABB(parent), expand() is monotone down
the tree, so F is exactly the set of non-expanded nodes whose ancestors all
expand (what a top-down traversal visits). ``cut_topdown`` computes that
traversal literally for small trees; the tests check the two agree.
"""
from __future__ import annotations

import numpy as np

NEAR_REL = 1e-6   # relative margin under which a predicate decision is "near threshold"


def frustum_planes(cam):
    """Five half-spaces {x : n . (x - pos) >= d} in world coordinates, FP64.

    Side planes pass through the camera centre: in camera coordinates the
    left/right/top/bottom image edges are fx*x + cx*z >= 0,
    -fx*x + (W - cx)*z >= 0, fy*y + cy*z >= 0 and -fy*y + (H - cy)*z >= 0; the
    near plane is z >= near. With x_cam = R (x - pos) a camera-space normal n_c
    becomes the world normal R^T n_c."""
    R = np.asarray(cam.R, np.float64)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    W, H = float(cam.width), float(cam.height)
    nc = np.array([[fx, 0.0, cx], [-fx, 0.0, W - cx], [0.0, fy, cy], [0.0, -fy, H - cy], [0.0, 0.0, 1.0]])
    nw = np.einsum("ij,jk->ik", nc, R)   # row i = (R^T nc_i)^T; einsum, not BLAS (see predicates)
    d = np.array([0.0, 0.0, 0.0, 0.0, float(np.float32(cam.near))])
    return nw, d


def predicates(scene, cam, tau: float, ids=None):
    """vis, ext, dist, expand and near-threshold flags for nodes `ids` (all by default)."""
    ids = np.arange(scene.n_nodes) if ids is None else np.asarray(ids)
    lo = scene.aabb_lo[ids].astype(np.float64)
    hi = scene.aabb_hi[ids].astype(np.float64)
    pos = np.asarray(cam.pos, np.float64)
    nw, d = frustum_planes(cam)
    vis = np.ones(len(ids), bool)
    near_plane = np.zeros(len(ids), bool)
    for k in range(5):
        n = nw[k]
        pv = np.where(n >= 0, hi, lo)
        # dot products as einsum sums (numpy's own loops): predicates_threaded
        # runs this on several threads, and numpy's threaded OpenBLAS has
        # returned wrong products to concurrent callers
        s = np.einsum("nj,j->n", pv - pos, n) - d[k]
        scale = np.einsum("nj,j->n", np.abs(pv - pos), np.abs(n)) + abs(d[k])
        vis &= s >= 0
        near_plane |= np.abs(s) <= NEAR_REL * scale
    ext = np.max(hi - lo, axis=1)
    dd = np.maximum(np.maximum(lo - pos, pos - hi), 0.0)
    dist = np.sqrt(np.sum(dd * dd, axis=1))
    f = float(np.float32(cam.fx))
    lhs = f * ext
    rhs = float(tau) * dist
    internal = scene.child_count[ids] > 0
    expand = internal & vis & (lhs > rhs)
    near_tau = np.abs(lhs - rhs) <= NEAR_REL * np.maximum(lhs, rhs)
    return dict(vis=vis, ext=ext, dist=dist, expand=expand, internal=internal,
                near=near_plane | (near_tau & internal), near_plane=near_plane,
                near_tau=near_tau & internal)


def predicates_threaded(scene, cam, tau: float, threads: int = 1, chunk: int = 1 << 21):
    """predicates() over all nodes, evaluated in chunks of nodes on `threads`
    threads (numpy releases the GIL in its array loops). Per-node arithmetic
    is that of predicates(); only the work is split."""
    N = scene.n_nodes
    if threads <= 1 or N <= chunk:
        return predicates(scene, cam, tau)
    from concurrent.futures import ThreadPoolExecutor
    starts = list(range(0, N, chunk))
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda a: predicates(scene, cam, tau, np.arange(a, min(N, a + chunk))), starts))
    return {k: np.concatenate([q[k] for q in parts]) for k in parts[0]}


def cut_bruteforce(scene, cam, tau: float, threads: int = 1):
    """Frontier F and cut C as sorted int64 node ids, plus the predicate table.

    Brute force over every node: n is in F iff not expand(n) and (n is the
    root or expand(parent(n))); C = F with vis."""
    P = predicates_threaded(scene, cam, tau, threads)
    e = P["expand"]
    par = scene.parent
    parent_exp = np.where(par >= 0, e[np.maximum(par, 0)], True)
    inF = (~e) & parent_exp
    F = np.nonzero(inF)[0]
    C = F[P["vis"][F]]
    return F, C, P


def cut_topdown(scene, cam, tau: float):
    """Literal top-down traversal from the root (pure Python; small trees only)."""
    P = predicates(scene, cam, tau)
    F, stack = [], [0]
    while stack:
        n = stack.pop()
        if P["expand"][n]:
            fc, cc = int(scene.first_child[n]), int(scene.child_count[n])
            stack.extend(range(fc, fc + cc))
        else:
            F.append(n)
    F = np.array(sorted(F), dtype=np.int64)
    C = F[P["vis"][F]]
    return F, C


def levels(scene):
    """Node ids grouped by depth (root first), from first_child/child_count."""
    out, cur = [], np.array([0], np.int64)
    while len(cur):
        out.append(cur)
        cc = scene.child_count[cur].astype(np.int64)
        internal = cur[cc > 0]
        if not len(internal):
            break
        fc = scene.first_child[internal].astype(np.int64)
        cnt = scene.child_count[internal].astype(np.int64)
        starts = np.repeat(fc, cnt)
        offs = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        cur = np.sort(starts + offs)
    return out


def ancestors_of(scene, nodes) -> np.ndarray:
    """Sorted ids of all strict ancestors of `nodes` (vectorised, level by level)."""
    N = scene.n_nodes
    mark = np.zeros(N, bool)
    cur = np.unique(np.asarray(nodes, np.int64))
    while len(cur):
        p = scene.parent[cur].astype(np.int64)
        p = np.unique(p[p >= 0])
        p = p[~mark[p]]
        mark[p] = True
        cur = p
    return np.nonzero(mark)[0]


def check_frontier(scene, F) -> bool:
    """Every root-to-leaf path holds exactly one node of F (antichain + cover)."""
    N = scene.n_nodes
    count = np.zeros(N, np.int64)     # number of F nodes on the path root..n
    inF = np.zeros(N, bool)
    inF[np.asarray(F, np.int64)] = True
    for lev in levels(scene):
        p = scene.parent[lev]
        count[lev] = np.where(p >= 0, count[np.maximum(p, 0)], 0) + inF[lev]
    leaves = scene.child_count == 0
    return bool(np.all(count[leaves] == 1))


def compare_cut(scene, cam, tau, F_gpu, C_gpu, oracle=None, threads=1):
    """Compare a GPU cut with the brute-force one.

    The expanded sets (strict ancestors of each frontier) may differ only in
    near-threshold nodes; cut differences must be explained by those or by a
    near-threshold frustum test. Returns a dict with counts and `ok`."""
    F_or, C_or, P = oracle if oracle is not None else cut_bruteforce(scene, cam, tau, threads)
    F_gpu = np.asarray(F_gpu, np.int64)
    C_gpu = np.asarray(C_gpu, np.int64)
    E_gpu = ancestors_of(scene, F_gpu)
    E_or = ancestors_of(scene, F_or)
    res = {}
    dE = np.setxor1d(E_gpu, E_or)
    bad_E = dE[~P["near"][dE]]
    res.update(expand_diff=int(len(dE)), expand_diff_unexplained=int(len(bad_E)))
    dF = np.setxor1d(F_gpu, F_or)
    dC = np.setxor1d(C_gpu, C_or)
    # a cut difference is explained if the node's frontier membership differs
    # (caused by an explained expand difference) or its vis test is near threshold
    explained = np.isin(dC, dF) | P["near_plane"][dC]
    # frontier differences must be children of differing expanded nodes
    par = scene.parent[dF] if len(dF) else np.zeros(0, np.int64)
    f_explained = np.isin(par, dE) | np.isin(dF, dE)
    res.update(F_size=int(len(F_gpu)), C_size=int(len(C_gpu)), F_diff=int(len(dF)), C_diff=int(len(dC)),
               C_diff_unexplained=int(np.sum(~explained)),
               F_diff_unexplained=int(np.sum(~f_explained)),
               near_nodes=int(np.sum(P["near"])))
    res["ok"] = (res["expand_diff_unexplained"] == 0 and res["C_diff_unexplained"] == 0
                 and res["F_diff_unexplained"] == 0)
    return res
