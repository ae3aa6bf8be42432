"""Input generator checks (CPU only): determinism, tree structure, fp32 AABB
containment (what makes the LoD predicate monotone), and the leaf recipe."""
import numpy as np

import scenegen


def test_deterministic_and_structure():
    cfg = scenegen.scaled_config("tiny", 3000)
    a = scenegen.make_city(cfg)
    b = scenegen.make_city(cfg)
    for k in ("mean", "log_scale", "quat", "opacity_logit", "sh", "aabb_lo", "aabb_hi", "parent", "first_child"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    N = a.n_nodes
    assert N == 2 * 3000 - 1 and a.parent[0] == -1
    ch = np.arange(1, N)
    assert np.all(a.parent[ch] < ch)                          # BFS: parents precede children
    internal = np.nonzero(a.child_count > 0)[0]
    assert np.all(a.child_count[internal] == 2)
    fc = a.first_child[internal]
    assert np.all(a.parent[fc] == internal) and np.all(a.parent[fc + 1] == internal)
    assert np.all(a.aabb_lo[ch] >= a.aabb_lo[a.parent[ch]]) and np.all(a.aabb_hi[ch] <= a.aabb_hi[a.parent[ch]])
    assert np.all(a.aabb_lo <= a.mean) and np.all(a.mean <= a.aabb_hi)
    np.testing.assert_allclose(np.linalg.norm(a.quat, axis=1), 1.0, atol=1e-5)
    # levels are contiguous id ranges
    ls = a.level_start
    assert ls[0] == 0 and ls[-1] == N


def test_leaf_recipe_statistics():
    cfg = scenegen.scaled_config("tiny", 20000)
    L = scenegen.generate_leaves(cfg)
    ls = L["log_scale"].astype(float)
    assert abs(ls.mean() - np.log(0.3)) < 0.02 and abs(ls.std() - 0.5) < 0.02
    assert abs(L["opacity_logit"].std() - 1.5) < 0.05
    sh = L["sh"].astype(float)
    assert abs(sh[:, 0, :].mean() - 0.5) < 0.01 and abs(sh[:, 1:, :].std() - 0.2) < 0.01
    ground = L["mean"][:, 2] == 0
    assert 0.45 < ground.mean() < 0.55
    assert np.all(np.abs(L["mean"][:, :2]) <= cfg.extent / 2 + 40)
