"""CPU pins of the brute-force adaptive-tree reference (tests/adaptive_ref.py).

The reference defines U, V, W and X pair by pair from Section 6 (refine while a box holds more
than N_leaf points) and the Carrier-Greengard-Rokhlin definitions.  What fixes it independently
of those definitions is the property the lists exist for: summed over U, and over V, W and X of
the target's ancestors, every (target leaf, source leaf) pair is counted exactly once.  The
tests check that on clustered point sets whose leaves spread over many levels, that the
property fails when a list is dropped (so the check sees such a mistake), and that a uniform
tree gives the lists of Definition 6.1 (no W or X, V = the interaction lists).
"""
import numpy as np
import pytest

import adaptive_ref as ar


def _clustered(seed, n, D, ncl=4, sigma=6.0):
    rng = np.random.default_rng(seed)
    side = 1 << D
    centres = rng.uniform(0.2 * side, 0.8 * side, size=(ncl, 2))
    pts = set()
    while len(pts) < n:
        c = centres[rng.integers(ncl)]
        scale = sigma * (1.0 + 20.0 * rng.random() ** 4)   # dense cores and wide tails
        p = np.clip(np.rint(c + scale * rng.standard_normal(2)), 0, side - 1).astype(int)
        pts.add((int(p[0]), int(p[1])))
    return np.array(sorted(pts), dtype=np.int64)


def _tree(xy, D, max_leaf, direct_max=None):
    L = 0
    while True:   # leaf level: the smallest at which no box holds more than max_leaf points
        _, c = np.unique(xy >> (D - L), axis=0, return_counts=True)
        if c.max() <= max_leaf or L == D:
            break
        L += 1
    level, x, y, parent, count = ar.uniform_tree(xy, D, L)
    role = ar.roles(level, parent, count, max_leaf, L)
    inst = np.zeros(len(level), dtype=np.int64)
    U, V, W, X = ar.lists(level, x, y, parent, inst, role, count, direct_max)
    return dict(level=level, x=x, y=y, parent=parent, count=count, role=role, inst=inst, U=U, V=V, W=W, X=X, L=L)


@pytest.mark.parametrize("seed,n,D,max_leaf", [(1, 400, 9, 4), (2, 700, 10, 8), (3, 300, 12, 2)])
def test_every_pair_counted_once(seed, n, D, max_leaf):
    t = _tree(_clustered(seed, n, D), D, max_leaf)
    leaf_levels = set(t["level"][t["role"] == ar.LEAF].tolist())
    assert len(leaf_levels) >= 3          # a genuinely adaptive tree
    assert sum(len(w) for w in t["W"]) > 0 and sum(len(x) for x in t["X"]) > 0
    cov = ar.coverage(t["parent"], t["role"], t["U"], t["V"], t["W"], t["X"], t["inst"])
    assert cov and set(cov.values()) == {1}
    # the leaves partition the points
    assert t["count"][t["role"] == ar.LEAF].sum() == n


@pytest.mark.parametrize("seed,n,D,max_leaf,direct_max", [(1, 400, 9, 4, 6), (2, 700, 10, 8, 12),
                                                          (4, 900, 11, 4, 48)])
def test_direct_rule_keeps_every_pair_counted_once(seed, n, D, max_leaf, direct_max):
    t = _tree(_clustered(seed, n, D), D, max_leaf, direct_max)
    base = _tree(_clustered(seed, n, D), D, max_leaf)
    # the rule only moves work: fewer W and X entries, more U entries
    assert sum(map(len, t["W"])) < sum(map(len, base["W"]))
    assert sum(map(len, t["X"])) < sum(map(len, base["X"]))
    assert sum(map(len, t["U"])) > sum(map(len, base["U"]))
    small = t["count"] <= direct_max
    assert all(not small[d] for w in t["W"] for d in w)
    assert all(len(t["X"][b]) == 0 for b in np.nonzero(small)[0])
    cov = ar.coverage(t["parent"], t["role"], t["U"], t["V"], t["W"], t["X"], t["inst"])
    assert set(cov.values()) == {1}


@pytest.mark.parametrize("drop", ["U", "V", "W", "X"])
def test_coverage_detects_a_missing_list(drop):
    t = _tree(_clustered(2, 700, 10), 10, 8)
    lists = {k: t[k] for k in "UVWX"}
    lists[drop] = [[] for _ in lists[drop]]
    cov = ar.coverage(t["parent"], t["role"], lists["U"], lists["V"], lists["W"], lists["X"], t["inst"])
    assert min(cov.values()) == 0


def test_uniform_tree_has_no_w_or_x():
    # every cell of a 32 x 32 grid, N_leaf 4: boxes of 2 x 2 cells hold 4 points and every
    # coarser box more, so all leaves sit on the finest level (level 4)
    D = 5
    g = np.arange(1 << D)
    xy = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    t = _tree(xy, D, 4)
    level, role = t["level"], t["role"]
    assert t["L"] == 4 and set(level[role == ar.LEAF].tolist()) == {4}
    assert all(len(w) == 0 for w in t["W"]) and all(len(x) == 0 for x in t["X"])
    # V of every box of level >= 2: the same-level boxes in the 6 x 6 block of its parent's
    # neighbourhood that are not its neighbours (Definition 6.1): 27 away from the edges
    for b in np.nonzero(level >= 2)[0]:
        lb, xb, yb = level[b], t["x"][b], t["y"][b]
        expect = []
        for c in np.nonzero(level == lb)[0]:
            dx, dy = t["x"][c] - xb, t["y"][c] - yb
            px, py = (t["x"][c] >> 1) - (xb >> 1), (t["y"][c] >> 1) - (yb >> 1)
            if max(abs(dx), abs(dy)) >= 2 and max(abs(px), abs(py)) <= 1:
                expect.append(int(c))
        assert t["V"][b] == sorted(expect)
        inner = 2 <= xb >> 1 << 1 and (xb | 1) + 2 < (1 << lb) and 2 <= yb >> 1 << 1 and (yb | 1) + 2 < (1 << lb)
        if inner:
            assert len(expect) == 27
    cov = ar.coverage(t["parent"], role, t["U"], t["V"], t["W"], t["X"], t["inst"])
    assert set(cov.values()) == {1}
