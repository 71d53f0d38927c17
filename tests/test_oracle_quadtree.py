"""Pins of the quadtree oracle (Sec. 6.1-6.3: quadtree partition, refinement, 4d partition)."""

import numpy as np
import pytest

from oracle import quadtree as qt
from oracle import region_adapt as ra


def _points(n, seed, skew=3.0):
    rng = np.random.default_rng(seed)
    return rng.random(n) ** skew, rng.random(n)


def _grow(forest, rounds, n, m_split, seed, state=None):
    splits = 0
    for r in range(rounds):
        x, y = _points(n, seed + r)
        roots = np.random.default_rng(seed + 100 + r).integers(0, forest.n_roots, n)
        for rt, a, b in zip(roots.tolist(), x.tolist(), y.tolist()):
            forest.lookup(rt, a, b)
        splits += forest.refine(m_split, state)
    return splits


def test_leaf_count_and_area_are_conserved():
    f = qt.Forest(n_roots=3, capacity=10_000)
    splits = _grow(f, rounds=5, n=4000, m_split=200, seed=1)
    assert splits > 10
    assert len(f.leaves()) == 3 + 3 * splits          # each split turns 1 leaf into 4
    assert f.area() == pytest.approx(3.0, abs=1e-15)  # the leaves tile every tree
    assert len(f.nodes) == 3 + 4 * splits


def test_lookup_is_the_containing_leaf():
    # descent agrees with a brute-force search over all leaves of the tree
    f = qt.Forest(n_roots=2, capacity=5000)
    _grow(f, rounds=4, n=3000, m_split=100, seed=2)
    roots_of = {}
    for n in f.nodes:  # root of every node, from the child links
        if n.index < f.n_roots:
            roots_of[n.index] = n.index
        if n.children:
            for c in n.children:
                roots_of[c.index] = roots_of[n.index]
    rng = np.random.default_rng(3)
    for _ in range(500):
        rt, x, y = int(rng.integers(0, 2)), float(rng.random()), float(rng.random())
        got = f.lookup(rt, x, y, count=False)
        want = [n.index for n in f.leaves() if roots_of[n.index] == rt
                and n.x0 <= x < n.x0 + n.side and n.y0 <= y < n.y0 + n.side]
        assert want == [got]
    # boundary and invalid points
    assert f.lookup(0, 1.0, 1.0, count=False) >= 0
    for rt, x, y in [(0, -0.1, 0.5), (0, 0.5, 1.5), (0, float("nan"), 0.2), (5, 0.5, 0.5), (-1, 0.5, 0.5)]:
        assert f.lookup(rt, x, y, count=False) == -1


def test_refinement_rule():
    f = qt.Forest(n_roots=1, capacity=100)
    for _ in range(11):
        f.lookup(0, 0.1, 0.1)
    assert f.refine(10) == 1                      # 11 visits > M_split = 10: split
    assert f.child_array() == [1, -1, -1, -1, -1] and f.depth_array() == [0, 1, 1, 1, 1]
    assert all(n.visits == 0 for n in f.nodes)    # counters restart
    for _ in range(10):
        f.lookup(0, 0.1, 0.1)                     # leaf 1 (lower-left quadrant)
    assert f.refine(10) == 0                      # exactly M_split visits: no split
    for _ in range(11):
        f.lookup(0, 0.9, 0.1)                     # leaf 2: x >= 1/2, y < 1/2
    assert f.refine(10) == 1
    assert f.child_array()[2] == 5 and f.nodes[5].x0 == 0.5 and f.nodes[8].y0 == 0.25


def test_children_inherit_parameters():
    state = ra.initial_state(100)
    state["lambda"][0] = -2.5
    state["updates"][0] = 11
    state["acc"][0] = 3.0
    f = qt.Forest(n_roots=1, capacity=100)
    for _ in range(6):
        f.lookup(0, 0.3, 0.7)
    f.refine(5, state)
    assert state["lambda"][1:5].tolist() == [-2.5] * 4
    assert state["updates"][1:5].tolist() == [2] * 4   # floor(11 / 4)
    assert state["acc"][1:5].tolist() == [0.0] * 4
    state["updates"][3] = 2
    for _ in range(6):
        f.lookup(0, 0.3, 0.7)                        # quadrant 2 of the root: node 3
    f.refine(5, state)
    assert state["updates"][5:9].tolist() == [1] * 4   # floor(2 / 4) = 0, kept >= 1


def test_capacity_limits_splits_in_node_order():
    f = qt.Forest(n_roots=4, capacity=12)          # room for two splits
    for rt in range(4):
        for _ in range(3):
            f.lookup(rt, 0.5, 0.5)
    assert f.refine(2) == 2
    assert f.child_array()[:4] == [4, 8, -1, -1]


def test_depth_limit():
    f = qt.Forest(n_roots=1, capacity=1000)
    for _ in range(qt.MAX_DEPTH + 3):
        for _ in range(2):
            f.lookup(0, 1e-9, 1e-9)
        f.refine(1)
    assert max(f.depth_array()) == qt.MAX_DEPTH


def test_vectorised_lookup_equals_pointer_descent():
    # the level-synchronous lookup_many is the per-point pointer descent, also at cell
    # corners, on the boundary x = 1 and for invalid points, and counts the same visits
    a = qt.Forest(n_roots=4, capacity=20_000)
    b = qt.Forest(n_roots=4, capacity=20_000)
    for r in range(5):
        rng = np.random.default_rng(50 + r)
        n = 3000
        x = (rng.random(n) ** 3).astype(np.float32)
        y = rng.random(n).astype(np.float32)
        x[:40] = np.round(x[:40] * 64) / 64            # exactly on cell corners
        y[40:60] = 1.0
        x[60] = np.nan
        y[61] = -0.25
        root = rng.integers(-1, 5, n)                  # includes -1 and 4 (invalid)
        got = a.lookup_many(root, x, y)
        want = [b.lookup(int(t), float(u), float(v)) for t, u, v in zip(root, x, y)]
        assert got.tolist() == want
        assert a.visits_array() == b.visits_array()
        assert a.refine(60) == b.refine(60)
    assert a.child_array() == b.child_array()
    assert len(a.nodes) > 100
