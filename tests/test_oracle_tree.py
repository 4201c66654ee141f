"""Pins for the oracle's root cube, keys, octree and interaction lists (CPU only)."""
import os

import numpy as np
import pytest

import workloads
from oracle import tree as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "morton_keys.txt")


def _golden_keys():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            a = line.split()
            rows.append(([float(a[0]), float(a[1]), float(a[2])], int(a[3])))
    return rows


def test_keys_match_hand_computed_fixture():
    rows = _golden_keys()
    x = np.array([r[0] for r in rows])
    k = T.morton(T.quantise(x, np.zeros(3), 1.0))
    assert [int(v) for v in k] == [r[1] for r in rows]


def test_root_box_automatic():
    x = np.array([[0.1, 0.2, 0.3], [0.7, 0.25, 0.35]])
    lo, s = T.root_box(x)
    assert s == 1.0                              # extent 0.6 -> next power of two
    np.testing.assert_array_equal(lo, np.floor(np.array([0.1, 0.2, 0.3]) * 4096) / 4096)
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.1, 0.1]])
    lo, s = T.root_box(x)
    assert s == 1.0                              # 0.5 (1 + 2^-10) > 0.5
    x = np.array([[0.0, 0.0, 0.0], [0.25, 0.1, 0.1]])
    assert T.root_box(x)[1] == 0.5
    with pytest.raises(ValueError):
        T.root_box(np.array([[0.0, 0.0, 2.0]]), ((0, 0, 0), 1.0))
    with pytest.raises(ValueError):
        T.root_box(np.array([[0.0, 0.0, 0.5]]), ((0, 0, 0), 3.0))
    with pytest.raises(ValueError):
        T.root_box(np.array([[np.nan, 0.0, 0.5]]))


def test_sort_is_stable_by_key_then_index():
    rng = np.random.default_rng(0)
    x = np.round(rng.random((3000, 3)) * 8) / 8      # many coincident keys
    t = T.build_tree(x, 16, True, 21, ((0, 0, 0), 1.0))
    keys = T.morton(T.quantise(x, np.zeros(3), 1.0))
    ref = np.lexsort((np.arange(3000), keys))
    np.testing.assert_array_equal(t.perm, ref)


@pytest.mark.parametrize("k,n,leaf", [(1, 4096, 64), (2, 20000, 64), (5, 20000, 32)])
def test_tree_invariants(k, n, leaf):
    w = workloads.make(k, n=n)
    t = T.build_tree(w.positions, leaf, w.adaptive, w.max_depth, w.root)
    # every point in exactly one leaf
    cover = np.zeros(n, dtype=int)
    for b in t.leaves():
        cover[t.begin[b]:t.end[b]] += 1
    assert np.all(cover == 1)
    for b in range(t.nboxes):
        assert t.end[b] > t.begin[b]
        if t.is_leaf[b]:
            if w.adaptive:
                assert t.end[b] - t.begin[b] <= leaf or t.level[b] == w.max_depth
        else:
            ch = t.children[b][t.children[b] >= 0]
            assert t.begin[ch].min() == t.begin[b] and t.end[ch].max() == t.end[b]
            assert np.sum(t.end[ch] - t.begin[ch]) == t.end[b] - t.begin[b]
            if w.adaptive:
                assert t.end[b] - t.begin[b] > leaf
        # points lie inside their box (integer cells)
        sh = T.BITS - t.level[b]
        k = T.quantise(w.positions[t.perm[t.begin[b]:t.end[b]]], t.lo, t.s) >> sh
        assert np.all(k == t.anchor[b])


def test_uniform_4096_shape():
    w = workloads.make(1)
    t = T.build_tree(w.positions, w.leaf_size, w.adaptive, w.max_depth, w.root)
    assert t.nboxes == 73 and t.is_leaf.sum() == 64 and t.depth == 2


def _all_ancestors(t, b):
    out = []
    while b >= 0:
        out.append(int(b))
        b = int(t.parent[b])
    return out


def _coverage(t, L):
    """For every (target leaf, source leaf) pair count the interaction paths."""
    leaves = t.leaves()
    pos = {int(b): i for i, b in enumerate(leaves)}
    cnt = np.zeros((len(leaves), len(leaves)), dtype=int)
    desc_leaves = {}

    def dl(a):
        if a not in desc_leaves:
            if t.is_leaf[a]:
                desc_leaves[a] = [a]
            else:
                desc_leaves[a] = [l for c in t.children[a] if c >= 0 for l in dl(int(c))]
        return desc_leaves[a]

    for B in leaves:
        B = int(B)
        i = pos[B]
        for A in L.U[B]:
            cnt[i, pos[A]] += 1
        for A in L.W[B]:
            for l in dl(A):
                cnt[i, pos[l]] += 1
        for anc in _all_ancestors(t, B):
            for A in L.V[anc]:
                for l in dl(A):
                    cnt[i, pos[l]] += 1
            for A in L.X[anc]:
                cnt[i, pos[A]] += 1
    return cnt


@pytest.mark.parametrize("k,n,leaf", [(1, 4096, 64), (2, 6000, 32), (5, 6000, 16)])
def test_lists_cover_every_pair_exactly_once(k, n, leaf):
    w = workloads.make(k, n=n)
    t = T.build_tree(w.positions, leaf, w.adaptive, w.max_depth, w.root)
    L = T.build_lists(t)
    cnt = _coverage(t, L)
    assert np.all(cnt == 1)


def test_list_definitions_by_brute_force():
    w = workloads.make(2, n=6000)
    t = T.build_tree(w.positions, 32, True, 21, w.root)
    L = T.build_lists(t)
    leaves = [int(b) for b in t.leaves()]
    assert sum(len(L.X[b]) for b in range(t.nboxes)) > 0      # the example is adaptive
    for B in leaves:
        ref = sorted(A for A in leaves if T.adjacent(t, A, B))
        assert L.U[B] == ref
    for B in range(t.nboxes):
        for A in L.V[B]:
            d = t.anchor[A] - t.anchor[B]
            assert t.level[A] == t.level[B] >= 2
            assert np.max(np.abs(d)) in (2, 3)
            T.v_offset_index(d)
        for A in L.X[B]:
            assert t.is_leaf[A] and t.level[A] < t.level[B]
            assert not T.adjacent(t, A, B) and T.adjacent(t, A, int(t.parent[B]))


def test_uniform_4096_list_counts_closed_form():
    # uniform depth 2: 64 leaves; adjacent pairs = (sum over a 4-cell axis of 3,2,2,3... ) ^3
    # per axis: cells 0..3 have 2,3,3,2 neighbours incl. self -> 10; 10^3 = 1000 U pairs;
    # every other ordered pair is a V pair: 64^2 - 1000 = 3096.
    w = workloads.make(1)
    t = T.build_tree(w.positions, w.leaf_size, w.adaptive, w.max_depth, w.root)
    L = T.build_lists(t)
    assert sum(len(u) for u in L.U) == 1000
    assert sum(len(v) for v in L.V) == 3096
    assert sum(len(x) for x in L.W) == 0 and sum(len(x) for x in L.X) == 0
