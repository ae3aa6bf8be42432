"""CPU checks of the subtree partition behind VY_CUT_CHUNKED
(vy_partition_plan, Section 4.1 "LoD Tree Partitioning"): subtrees of height
2 rooted at depths 0, 3, 6, ... in BFS order, stored subtree after subtree,
and chunks of consecutive subtrees of at most 2048 nodes, as few as the
contiguity constraint allows (checked against a dynamic program)."""
import numpy as np
import pytest

import scenegen


def _vy():
    vy = pytest.importorskip("paper_2506_02774_amd")
    try:
        vy.lib()
    except ImportError as e:
        pytest.fail(f"library not built: {e}")
    return vy


def _depth(parent):
    d = np.zeros(len(parent), np.int64)
    for i in range(1, len(parent)):
        d[i] = d[parent[i]] + 1
    return d


@pytest.mark.parametrize("n_leaf", [1, 2, 7, 5000, 20000])
def test_partition_plan(n_leaf):
    vy = _vy()
    host = scenegen.make_city(scenegen.scaled_config("tiny", n_leaf)) if n_leaf > 1 else \
        scenegen.tree_from_arrays([-1], [-1], [0], [[0, 0, 0]], [[1, 1, 1]])
    n = len(host.parent)
    P = vy.partition_plan(host.parent, host.first_child, host.child_count)
    d = _depth(host.parent)
    roots = np.nonzero(d % 3 == 0)[0]
    assert np.array_equal(P["sub_root"], roots)                 # BFS order of the roots
    # each node's subtree root is its ancestor at depth 3 * floor(depth / 3)
    anc = np.arange(n)
    for _ in range(2):
        up = d[anc] % 3 != 0
        anc = np.where(up, host.parent[anc], anc)
    assert np.array_equal(P["sub_root"][P["sub_of"]], anc)
    # subtree-major order: a permutation; each subtree's nodes contiguous, root first, parents before children
    assert np.array_equal(np.sort(P["local"]), np.arange(n))
    sizes = np.diff(P["sub_rec"])
    assert sizes.sum() == n and np.all(sizes >= 1) and np.all(sizes <= 7)
    s_of_pos = np.repeat(np.arange(len(sizes)), sizes)
    assert np.array_equal(s_of_pos[P["local"]], P["sub_of"])
    assert np.array_equal(P["local"][roots], P["sub_rec"][:-1])
    nonroot = d % 3 != 0
    assert np.all(P["local"][host.parent[nonroot]] < P["local"][nonroot])
    # chunks: consecutive subtrees, at most 2048 nodes, the fewest possible
    cs = P["chunk_sub"]
    assert cs[0] == 0 and cs[-1] == len(sizes) and np.all(np.diff(cs) > 0)
    csum = np.concatenate([[0], np.cumsum(sizes)])
    assert np.all(csum[cs[1:]] - csum[cs[:-1]] <= 2048)
    best = np.full(len(sizes) + 1, 1 << 30)
    best[0] = 0
    for i in range(1, len(sizes) + 1):
        j = np.searchsorted(csum, csum[i] - 2048, side="left")   # earliest start with sum <= 2048
        best[i] = best[j:i].min() + 1
    assert len(cs) - 1 == best[-1]


def test_partition_plan_refuses_bad_trees():
    vy = _vy()
    with pytest.raises(vy.VoyagerError):       # a child numbered before its parent
        vy.partition_plan([-1, 2, 0], [2, -1, 1], [1, 0, 1])
    with pytest.raises(vy.VoyagerError):       # the root is not node 0
        vy.partition_plan([1, -1], [-1, 0], [0, 1])
