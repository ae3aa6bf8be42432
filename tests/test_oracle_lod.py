"""Pins for oracle.lod (CPU only): hand-derived cut, brute force vs a literal
top-down traversal, the frontier invariant, limiting tau values, monotonicity
of the predicate, and the comparison helper catching a planted mistake."""
import json
import math
import os

import numpy as np
import pytest

import scenegen
from oracle import lod

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold_tree():
    g = json.load(open(os.path.join(GOLD, "lod_7node.json")))
    sc = scenegen.tree_from_arrays(g["parent"], g["first_child"], g["child_count"], g["aabb_lo"], g["aabb_hi"])
    c = g["camera"]
    cam = scenegen.look_camera(c["pos"], math.radians(c["yaw_deg"]), math.radians(c["pitch_deg"]),
                               c["width"], c["height"], c["fov_x_deg"])
    return g, sc, cam


def test_hand_derived_cut():
    g, sc, cam = _gold_tree()
    for tau_s, exp in g["expected"].items():
        F, C, _ = lod.cut_bruteforce(sc, cam, float(tau_s))
        assert F.tolist() == exp["F"], tau_s
        assert C.tolist() == exp["C"], tau_s
        F2, C2 = lod.cut_topdown(sc, cam, float(tau_s))
        assert F2.tolist() == exp["F"] and C2.tolist() == exp["C"]


def _random_cams(cfg, n, seed):
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        p = rng.uniform(-0.3, 0.3, 2) * cfg.extent
        cams.append(scenegen.look_camera([p[0], p[1], rng.uniform(1.0, 40.0)], rng.uniform(0, 2 * math.pi),
                                         rng.uniform(-0.5, 0.2), 256, 192))
    return cams


@pytest.mark.parametrize("tau", [0.0, 0.5, 2.0, 8.0, 64.0])
def test_bruteforce_equals_topdown(tiny_scene, tau):
    for cam in _random_cams(scenegen.CONFIGS["tiny"], 4, 7):
        F, C, _ = lod.cut_bruteforce(tiny_scene, cam, tau)
        F2, C2 = lod.cut_topdown(tiny_scene, cam, tau)
        assert np.array_equal(F, F2) and np.array_equal(C, C2)
        assert lod.check_frontier(tiny_scene, F)


def test_limits(tiny_scene, tiny_cams):
    # tau -> infinity: only nodes whose AABB contains the camera (dist = 0) expand;
    # from a camera outside the root box the cut is the root alone
    far = scenegen.look_camera([0.0, 0.0, 5000.0], 0.0, -1.2, 256, 256)
    F, C, P = lod.cut_bruteforce(tiny_scene, far, 1e30)
    assert F.tolist() == [0] and C.tolist() == [0]
    cam = tiny_cams[0]
    F, C, P = lod.cut_bruteforce(tiny_scene, cam, 1e30)
    E = lod.ancestors_of(tiny_scene, F)
    assert np.all(P["dist"][E] == 0.0) and len(E) > 0
    # tau = 0: every visible internal node expands, so F is the set of nodes
    # whose strict ancestors are all visible and which are leaves or invisible
    F, C, P = lod.cut_bruteforce(tiny_scene, cam, 0.0)
    vis = P["vis"]
    ok_anc = np.ones(tiny_scene.n_nodes, bool)
    for lev in lod.levels(tiny_scene):
        p = tiny_scene.parent[lev]
        ok_anc[lev] = np.where(p >= 0, ok_anc[np.maximum(p, 0)] & vis[np.maximum(p, 0)], True)
    expect = np.nonzero(ok_anc & ((tiny_scene.child_count == 0) | ~vis))[0]
    assert np.array_equal(F, expect)
    assert np.all(tiny_scene.child_count[C] == 0)


def test_monotone_predicate(tiny_scene):
    """expand(child) implies expand(parent): the property that makes the cut
    well defined and a temporal search exact."""
    for cam in _random_cams(scenegen.CONFIGS["tiny"], 6, 11):
        for tau in (0.7, 2.0, 9.0):
            e = lod.predicates(tiny_scene, cam, tau)["expand"]
            ch = np.nonzero(tiny_scene.parent >= 0)[0]
            assert not np.any(e[ch] & ~e[tiny_scene.parent[ch]])


def test_predicate_pieces_closed_form():
    """dist and ext against hand values; p-vertex visibility against corner enumeration."""
    g, sc, cam = _gold_tree()
    P = lod.predicates(sc, cam, 2.0)
    assert P["ext"][1] == 8.0 and P["ext"][0] == 190.0
    h = float(np.float32(1.7)) - 1.0        # camera height is stored as float32
    assert abs(P["dist"][1] - math.hypot(4.0, h)) < 1e-12
    assert abs(P["dist"][2] - h) < 1e-12
    # visibility by enumerating the 8 corners (a box is outside a half-space iff all corners are)
    nw, d = lod.frustum_planes(cam)
    for n in range(sc.n_nodes):
        lo, hi = sc.aabb_lo[n].astype(float), sc.aabb_hi[n].astype(float)
        corners = np.array([[(lo, hi)[i][0], (lo, hi)[j][1], (lo, hi)[k][2]]
                            for i in (0, 1) for j in (0, 1) for k in (0, 1)])
        vis = all(np.any((corners - cam.pos.astype(float)) @ nw[p] - d[p] >= 0) for p in range(5))
        assert vis == bool(P["vis"][n])


def test_compare_cut_catches_planted_mistake(tiny_scene, tiny_cams):
    cam = tiny_cams[3]
    F, C, P = lod.cut_bruteforce(tiny_scene, cam, 2.0)
    assert lod.compare_cut(tiny_scene, cam, 2.0, F, C)["ok"]
    # a frontier node replaced by its children (a wrong expansion)
    n = int(F[np.nonzero(tiny_scene.child_count[F] > 0)[0][0]]) if np.any(tiny_scene.child_count[F] > 0) else None
    if n is not None:
        fc = tiny_scene.first_child[n]
        F2 = np.sort(np.concatenate([F[F != n], [fc, fc + 1]]))
        C2 = F2[P["vis"][F2]]
        assert not lod.compare_cut(tiny_scene, cam, 2.0, F2, C2)["ok"]
    # a dropped cut node
    assert not lod.compare_cut(tiny_scene, cam, 2.0, F, C[1:])["ok"]
