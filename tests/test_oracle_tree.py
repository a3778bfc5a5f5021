"""Pins of the oracle's octree and interaction lists (see oracle/tree.py)."""

import os

import numpy as np
import pytest

import workloads as W
from oracle import tree as T

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold_lists():
    out = {}
    for line in open(os.path.join(GOLD, "uniform_depth3_lists.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = int(v)
    return out


def _cloud(seed, n_uniform=600, n_blob=900):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.random((n_uniform, 3)), 0.3 + 0.01 * rng.standard_normal((n_blob, 3))])
    return x.astype(np.float32)


def test_morton_interleave_small():
    q = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 0, 0], [2 ** 21 - 1] * 3])
    k = T.interleave(q)
    assert list(k[:4]) == [4, 2, 1, 4 + 32]
    assert int(k[4]) == 2 ** 63 - 1


def test_uniform_depth3_counts_match_hand_derivation():
    g = _gold_lists()
    d = W.cube_uniform()
    t = T.build_tree(d["xyz"], uniform_depth=3, root=d["root"])
    L = T.all_lists(t)
    assert len(t.level) == g["boxes"]
    assert int(t.leaf.sum()) == g["leaves"]
    assert sum(len(v) for v in L["U"].values()) == g["U"]
    v2 = sum(len(L["V"][b]) for b in range(len(t.level)) if t.level[b] == 2)
    v3 = sum(len(L["V"][b]) for b in range(len(t.level)) if t.level[b] == 3)
    assert (v2, v3) == (g["V_level2"], g["V_level3"])
    assert sum(len(v) for v in L["W"].values()) == g["W"]
    assert sum(len(v) for v in L["X"].values()) == g["X"]


@pytest.mark.parametrize("s", [8, 20, 64])
def test_points_belong_to_their_leaf_by_brute_force(s):
    x = _cloud(1)
    t = T.build_tree(x, leaf_size=s)
    x0, w = T.root_box(x)
    q = T.quantise(x, x0, w)
    leaves = np.flatnonzero(t.leaf)
    # brute force: which leaf cube contains each point (integer coordinates)
    lo = t.lo[leaves]
    hi = lo + t.size[leaves][:, None]
    inside = np.all((q[:, None, :] >= lo[None]) & (q[:, None, :] < hi[None]), axis=2)
    assert np.all(inside.sum(axis=1) == 1)
    owner = leaves[np.argmax(inside, axis=1)]
    for b in leaves:
        members = np.sort(t.order[t.begin[b]:t.end[b]])
        np.testing.assert_array_equal(members, np.flatnonzero(owner == b))
        assert t.end[b] - t.begin[b] <= s or t.level[b] == T.MAXLEV
    inner = np.flatnonzero(~t.leaf)
    assert np.all(t.end[inner] - t.begin[inner] > s)


def test_tree_invariant_under_input_permutation():
    x = _cloud(2)
    perm = np.random.default_rng(0).permutation(len(x))
    a = T.build_tree(x, leaf_size=16)
    b = T.build_tree(x[perm], leaf_size=16)
    for f in ("level", "begin", "end", "parent"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    np.testing.assert_array_equal(a.anchor, b.anchor)
    np.testing.assert_array_equal(a.keys, b.keys)


def test_tree_invariant_under_scaling_and_translation():
    x = _cloud(3).astype(np.float64)
    a = T.build_tree(x.astype(np.float32), leaf_size=16, root=(0.0, 0.0, 0.0, 1.0))
    y = (x * 4.0 + 8.0).astype(np.float32)  # exact in float32: power-of-two scale
    b = T.build_tree(y, leaf_size=16, root=(8.0, 8.0, 8.0, 4.0))
    for f in ("level", "begin", "end", "parent"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))


@pytest.mark.parametrize("seed,s", [(4, 12), (5, 30)])
def test_interaction_coverage_is_exactly_once(seed, s):
    t = T.build_tree(_cloud(seed), leaf_size=s)
    L = T.all_lists(t)
    assert sum(len(v) for v in L["W"].values()) > 0
    cnt = T.coverage(t, L)
    assert cnt.min() == 1 and cnt.max() == 1


def test_coverage_with_separate_targets_and_sources():
    rng = np.random.default_rng(9)
    trg = rng.random((400, 3)).astype(np.float32)
    src = (0.5 + 0.05 * rng.standard_normal((700, 3))).astype(np.float32)
    t = T.build_tree(src, trg=trg, leaf_size=25)
    assert t.tend[0] == 400 and t.send[0] == 700
    L = T.all_lists(t)
    cnt = T.coverage(t, L)
    assert cnt.min() == 1 and cnt.max() == 1
    np.testing.assert_array_equal(np.sort(t.trg_perm), np.arange(400))
    np.testing.assert_array_equal(np.sort(t.src_perm), np.arange(700))


def test_list_symmetries():
    t = T.build_tree(_cloud(6), leaf_size=15)
    L = T.all_lists(t)
    for b in range(len(t.level)):
        for a in L["U"][b]:
            assert b in L["U"][int(a)]
        for a in L["V"][b]:
            assert b in L["V"][int(a)]
        for a in L["W"][b]:
            assert b in L["X"][int(a)]


def test_degenerate_inputs():
    one = np.array([[0.3, 0.3, 0.3]], dtype=np.float32)
    t = T.build_tree(one, leaf_size=4)
    assert len(t.level) == 1 and t.leaf[0]
    same = np.full((50, 3), 0.25, dtype=np.float32)
    t = T.build_tree(same, leaf_size=8, max_depth=5)
    assert t.nlevels == 6 and t.end[-1] - t.begin[-1] == 50
    empty = np.zeros((0, 3), dtype=np.float32)
    t = T.build_tree(empty)
    assert len(t.level) == 0
