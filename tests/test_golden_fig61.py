"""The worked example after Definition 6.1 (Section 6), tests/golden/fig61_lists.txt, against the
brute-force tree reference (tests/adaptive_ref.py): a full four-level tree over an 8 x 8 grid of
points, N_leaf 1.  The interaction lists come from the reference's V definition; children and
neighbours from the uniform tree's parent links and the adjacency of Definition 6.1."""
import numpy as np

import adaptive_ref as ar
import golden_fixtures as gf


def _tree():
    g = np.arange(8)
    xy = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    level, x, y, parent, count = ar.uniform_tree(xy, 3, 3)
    role = ar.roles(level, parent, count, 1, 3)
    U, V, W, X = ar.lists(level, x, y, parent, np.zeros(len(level)), role)
    num = np.array([gf.paper_number(int(lv), int(a), int(b)) for lv, a, b in zip(level, x, y)])
    return level, x, y, parent, role, V, num


def test_example_lists():
    level, x, y, parent, role, V, num = _tree()
    assert sorted(num.tolist()) == list(range(1, 86))
    box = {int(n): i for i, n in enumerate(num)}
    assert set(level[role == ar.LEAF].tolist()) == {3}
    for (kind, b), expect in gf.fig61_lists().items():
        i = box[b]
        if kind == "child":
            got = [int(num[j]) for j in np.nonzero(parent == i)[0]]
        elif kind == "nei":
            same = np.nonzero(level == level[i])[0]
            got = [int(num[j]) for j in same
                   if j != i and max(abs(x[j] - x[i]), abs(y[j] - y[i])) == 1]
        else:
            got = [int(num[j]) for j in V[i]]
        assert sorted(got) == sorted(expect), (kind, b)
