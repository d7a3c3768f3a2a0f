"""Pins for the oracle's Morton order and octree lists.

The interleave is checked against a string-based construction; the lists
against brute-force geometry; and the partition property that makes the FMM
exact up to truncation: every ordered pair of leaves is covered exactly once,
either directly (U list) or by exactly one multipole-to-local (V list) pair
of ancestors.
"""
import itertools

import numpy as np

from oracle import tree
from workloads import cube_surface, icosphere


def test_interleave_matches_string_construction():
    rng = np.random.default_rng(0)
    for _ in range(200):
        q = [int(v) for v in rng.integers(0, 1 << 21, 3)]
        bits = [format(v, "021b") for v in q]
        s = "".join(bits[0][i] + bits[1][i] + bits[2][i] for i in range(21))
        assert tree.interleave(*q) == int(s, 2)
        assert tree.deinterleave(tree.interleave(*q)) == tuple(q)


def test_quantisation_bounds_and_order():
    V, T = icosphere(2)
    cen = V[T].mean(axis=1)
    q = np.array(tree.quantise(cen))
    assert q.min() >= 0 and q.max() <= tree.QMAX
    # monotone in each coordinate
    for a in range(3):
        o = np.argsort(cen[:, a], kind="stable")
        assert np.all(np.diff(q[o, a]) >= 0)
    keys = tree.morton_keys(cen)
    perm = tree.sort_order(keys)
    sk = [keys[i] for i in perm]
    assert sk == sorted(keys)
    # ties broken by original index
    for i in range(len(perm) - 1):
        if sk[i] == sk[i + 1]:
            assert perm[i] < perm[i + 1]


def _check_tree(t: tree.Tree):
    L = t.L
    # leaves partition the sorted elements
    assert t.leaf_start[0] == 0 and t.leaf_end[-1] == len(t.perm)
    assert all(e == s for e, s in zip(t.leaf_end[:-1], t.leaf_start[1:]))
    assert len(t.leaf_start) == len(t.boxes[L])
    leaves = t.boxes[L]
    anc = lambda b, l: b >> (3 * (L - l))
    vsets = {l: {b: set(t.vlist(l, b)) for b in t.boxes[l]} for l in range(2, L + 1)}
    for l in range(2, L + 1):
        for b, vs in vsets[l].items():
            bx = np.array(t.coords(b, l))
            for c in vs:
                cx = np.array(t.coords(c, l))
                d = np.abs(cx - bx).max()
                assert 2 <= d <= 3                       # well separated, parents adjacent
                assert b in vsets[l][c]                  # symmetric
    for A, B in itertools.product(leaves, leaves):
        direct = B in t.ulist(A)
        n_v = sum(anc(B, l) in vsets[l][anc(A, l)] for l in range(2, L + 1))
        assert direct + n_v == 1, (A, B, direct, n_v)


def test_tree_partition_property_sphere():
    V, T = icosphere(2)
    t = tree.Tree(V[T].mean(axis=1), leaf_cap=4)
    assert t.L >= 3
    _check_tree(t)


def test_tree_partition_property_cube():
    V, T = cube_surface(6)
    t = tree.Tree(V[T].mean(axis=1), leaf_cap=12)
    _check_tree(t)


def test_leaf_level_rule():
    V, T = icosphere(3)
    cen = V[T].mean(axis=1)
    t = tree.Tree(cen, leaf_cap=32)
    sh = 3 * (21 - t.L)
    counts = np.unique(np.array(t.sorted_keys, dtype=object) >> sh, return_counts=True)[1]
    assert counts.max() <= 32
    if t.L > 2:
        sh2 = 3 * (21 - (t.L - 1))
        counts2 = np.unique(np.array(t.sorted_keys, dtype=object) >> sh2, return_counts=True)[1]
        assert counts2.max() > 32
