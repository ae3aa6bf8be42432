"""GPU parity of the LoD cut (through the C ABI): the full search (worklist
traversal and exhaustive flat) against the FP64 brute-force oracle, and the
temporal search (Algorithm 1) bitwise equal to the full search from any seed."""
import numpy as np
import pytest

import scenegen
from oracle import lod as olod

from gpu_util import random_cameras, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny(tiny_scene):
    vy = require_gpu()
    return vy, vy.Scene(tiny_scene), tiny_scene


def test_scene_validates(tiny):
    vy, sc, host = tiny
    assert sc.validate() == 0


def test_full_cut_matches_oracle_walkthrough(tiny, tiny_cams):
    vy, sc, host = tiny
    for i, cam in enumerate(tiny_cams):
        for mode in (vy.VY_CUT_FRONTIER, vy.VY_CUT_FLAT):
            cut = vy.vy_lod_cut(sc, cam, 2.0, mode=mode)
            F, C = cut.ids()
            res = olod.compare_cut(host, cam, 2.0, F, C)
            print(f"frame {i} mode {mode}: {res}", flush=True)
            assert res["ok"], res
            assert olod.check_frontier(host, F)


def test_flat_equals_frontier_bitwise(tiny):
    vy, sc, host = tiny
    for cam in random_cameras(scenegen.CONFIGS["tiny"], 6, 21):
        for tau in (0.0, 0.7, 2.0, 16.0):
            a = vy.vy_lod_cut(sc, cam, tau, mode=vy.VY_CUT_FRONTIER).ids()
            b = vy.vy_lod_cut(sc, cam, tau, mode=vy.VY_CUT_FLAT).ids()
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_bfs_and_dfs_traversals_agree(tiny):
    """The workgroup breadth-first traversal (default) and the per-thread
    depth-first one give the same cut, bitwise, for full and temporal searches."""
    vy, sc, host = tiny
    cams = random_cameras(scenegen.CONFIGS["tiny"], 6, 41)
    for cam in cams:
        for tau in (0.0, 0.7, 2.0, 16.0):
            a = vy.vy_lod_cut(sc, cam, tau).ids()
            b = vy.vy_lod_cut(sc, cam, tau, mode=vy.VY_CUT_DFS).ids()
            c = vy.vy_lod_cut(sc, cam, tau, mode=vy.VY_CUT_FLAT).ids()
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    q, lv = vy.vy_lod_cut(sc, cams[0], 2.0), vy.vy_lod_cut(sc, cams[0], 2.0, mode=vy.VY_CUT_DFS)
    for cam in cams[1:]:
        q = vy.vy_lod_cut(sc, cam, 2.0, prev=q, out=q)
        lv = vy.vy_lod_cut(sc, cam, 2.0, prev=lv, out=lv, mode=vy.VY_CUT_DFS)
        a, b = q.ids(), lv.ids()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_traversals_on_a_larger_city():
    """200k leaves along a walkthrough: temporal == full (breadth-first) ==
    full (depth-first), and the full search matches the oracle."""
    vy = require_gpu()
    cfg = scenegen.scaled_config("med", 200_000)
    host = scenegen.make_city(cfg)
    sc = vy.Scene(host)
    cams = scenegen.walkthrough(cfg, frames=12, width=640, height=360)
    state = None
    for i, cam in enumerate(cams):
        state = vy.vy_lod_cut(sc, cam, 2.0, prev=state, out=state) if state is not None else vy.vy_lod_cut(sc, cam, 2.0)
        a = state.ids()
        b = vy.vy_lod_cut(sc, cam, 2.0).ids()
        c = vy.vy_lod_cut(sc, cam, 2.0, mode=vy.VY_CUT_DFS).ids()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), i
        assert np.array_equal(b[0], c[0]) and np.array_equal(b[1], c[1]), i
        if i % 6 == 0:
            res = olod.compare_cut(host, cam, 2.0, b[0], b[1])
            assert res["ok"], res


def test_temporal_equals_full_along_walkthrough(tiny, tiny_cams):
    vy, sc, host = tiny
    state = vy.vy_lod_cut(sc, tiny_cams[0], 2.0)
    for cam in tiny_cams[1:]:
        state = vy.vy_lod_cut(sc, cam, 2.0, prev=state, out=state)     # prev == out
        full = vy.vy_lod_cut(sc, cam, 2.0)
        a, b = state.ids(), full.ids()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_temporal_from_arbitrary_frontiers(tiny):
    vy, sc, host = tiny
    rng = np.random.default_rng(5)
    leaves = np.nonzero(host.child_count == 0)[0]
    seeds = {"root": np.array([0]), "leaves": leaves}
    # random valid frontier: cut of a random camera at a random tau
    cams = random_cameras(scenegen.CONFIGS["tiny"], 4, 33)
    seeds["other_camera"] = vy.vy_lod_cut(sc, cams[0], 7.0).ids()[0]
    for name, F0 in seeds.items():
        for cam in cams[1:]:
            for tau in (0.5, 2.0, 9.0):
                st = vy.Cut(sc)
                st.set_frontier(F0)
                out = vy.Cut(sc)
                vy.vy_lod_cut(sc, cam, tau, prev=st, out=out)
                full = vy.vy_lod_cut(sc, cam, tau)
                a, b = out.ids(), full.ids()
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (name, tau)


def test_cut_edge_cases(tiny):
    vy, sc, host = tiny
    # camera far above looking away (sky): nothing visible, F = {root} or a culled frontier
    cam = scenegen.look_camera([0.0, 0.0, 5000.0], 0.0, 1.2, 64, 64)
    F, C = vy.vy_lod_cut(sc, cam, 2.0).ids()
    res = olod.compare_cut(host, cam, 2.0, F, C)
    assert res["ok"] and len(C) == 0
    # tau = 0 from the street: visible leaves
    cam = scenegen.walkthrough(scenegen.CONFIGS["tiny"])[0]
    F, C = vy.vy_lod_cut(sc, cam, 0.0).ids()
    assert np.all(host.child_count[C] == 0)
    assert olod.compare_cut(host, cam, 0.0, F, C)["ok"]
    # huge tau from outside the root box: the root alone
    cam = scenegen.look_camera([0.0, 0.0, 5000.0], 0.0, -1.2, 64, 64)
    F, C = vy.vy_lod_cut(sc, cam, 1e30).ids()
    assert F.tolist() == [0] and C.tolist() == [0]


def test_single_node_scene():
    vy = require_gpu()
    host = scenegen.tree_from_arrays([-1], [-1], [0], [[-1, -1, 4]], [[1, 1, 6]], mean=[[0, 0, 5]])
    sc = vy.Scene(host)
    cam = scenegen.identity_camera(32, 32)
    F, C = vy.vy_lod_cut(sc, cam, 1.0).ids()
    assert F.tolist() == [0] and C.tolist() == [0]
    st = vy.vy_lod_cut(sc, cam, 1.0)
    F2, C2 = vy.vy_lod_cut(sc, cam, 1.0, prev=st, out=st).ids()
    assert F2.tolist() == [0] and C2.tolist() == [0]


def test_errors(tiny):
    vy, sc, host = tiny
    fresh = vy.Cut(sc)
    cam = scenegen.identity_camera(32, 32)
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_lod_cut(sc, cam, 1.0, prev=fresh)
    assert e.value.code == vy.VY_ERR_STATE
    other = vy.Scene(scenegen.make_city(scenegen.scaled_config("tiny", 500)))
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_lod_cut(other, cam, 1.0, out=vy.Cut(sc))
    assert e.value.code == vy.VY_ERR_ARG
    with pytest.raises(vy.VoyagerError):
        vy.vy_lod_cut(sc, cam, -1.0)


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_chunked_traversal_agrees(tiny):
    """VY_CUT_CHUNKED (Section 4.1: streamed chunks of height-2 subtrees for a
    full search, Algorithm 1 per subtree with TOP/BOTTOM for a temporal one)
    gives the default cut bit for bit: full searches, temporal searches along
    camera changes, and temporal searches from arbitrary frontiers."""
    vy, sc, host = tiny
    sc.partition()
    C = vy.VY_CUT_CHUNKED
    cams = random_cameras(scenegen.CONFIGS["tiny"], 6, 41)
    for cam in cams:
        for tau in (0.0, 0.7, 2.0, 16.0, 1e30):
            assert _same(vy.vy_lod_cut(sc, cam, tau, mode=C).ids(), vy.vy_lod_cut(sc, cam, tau).ids()), tau
    q = vy.vy_lod_cut(sc, cams[0], 2.0, mode=C)
    for cam in cams[1:] + cams[:2]:
        q = vy.vy_lod_cut(sc, cam, 2.0, prev=q, out=q, mode=C)
        assert _same(q.ids(), vy.vy_lod_cut(sc, cam, 2.0).ids())
    leaves = np.nonzero(host.child_count == 0)[0]
    seeds = {"root": np.array([0]), "leaves": leaves, "other": vy.vy_lod_cut(sc, cams[0], 7.0).ids()[0]}
    for name, F0 in seeds.items():
        for cam in cams[1:4]:
            for tau in (0.5, 2.0, 9.0):
                st = vy.Cut(sc)
                st.set_frontier(F0)
                out = vy.vy_lod_cut(sc, cam, tau, prev=st, mode=C)
                assert _same(out.ids(), vy.vy_lod_cut(sc, cam, tau).ids()), (name, tau)


def test_chunked_traversal_on_a_larger_city():
    vy = require_gpu()
    cfg = scenegen.scaled_config("med", 200_000)
    host = scenegen.make_city(cfg)
    sc = vy.Scene(host)
    sc.partition()
    cams = scenegen.walkthrough(cfg, frames=12, width=640, height=360)
    state = None
    for i, cam in enumerate(cams):
        state = vy.vy_lod_cut(sc, cam, 2.0, prev=state, out=state, mode=vy.VY_CUT_CHUNKED) if state is not None \
            else vy.vy_lod_cut(sc, cam, 2.0, mode=vy.VY_CUT_CHUNKED)
        a = state.ids()
        b = vy.vy_lod_cut(sc, cam, 2.0).ids()
        c = vy.vy_lod_cut(sc, cam, 2.0, mode=vy.VY_CUT_CHUNKED).ids()
        assert _same(a, b) and _same(b, c), i


def test_chunked_mode_errors(tiny):
    vy, sc, host = tiny
    cam = scenegen.identity_camera(32, 32)
    fresh = vy.Scene(scenegen.make_city(scenegen.scaled_config("tiny", 500)))
    with pytest.raises(vy.VoyagerError) as e:          # no partition
        vy.vy_lod_cut(fresh, cam, 1.0, mode=vy.VY_CUT_CHUNKED)
    assert e.value.code == vy.VY_ERR_STATE
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_lod_cut(sc, cam, 1.0, mode=vy.VY_CUT_CHUNKED | vy.VY_CUT_DFS)
    assert e.value.code == vy.VY_ERR_ARG
    one = vy.Scene(scenegen.tree_from_arrays([-1], [-1], [0], [[-1, -1, 4]], [[1, 1, 6]], mean=[[0, 0, 5]]))
    one.partition()
    F, C = vy.vy_lod_cut(one, scenegen.identity_camera(32, 32), 1.0, mode=vy.VY_CUT_CHUNKED).ids()
    assert F.tolist() == [0] and C.tolist() == [0]
