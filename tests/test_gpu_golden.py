"""The library's tree and lists against the worked example after Definition 6.1 (Section 6,
tests/golden/fig61_lists.txt): a plan over the 64 cells of an 8 x 8 grid with N_leaf 1 has the
four levels of Fig. 6.1; its exported children, neighbour and interaction lists, renumbered as
the fixture reads the figure, equal the printed ones."""
import numpy as np
import pytest

import adaptive_ref as ar
import golden_fixtures as gf

pytestmark = pytest.mark.gpu


def test_fig61_lists():
    import torch
    import paper_1105_3505_amd as lf
    g = np.arange(8, dtype=np.int32)
    xy = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2).copy()
    ctx = lf.Context(0, max_leaf=1)
    plan = ctx.plan(torch.from_numpy(xy).cuda())
    assert plan.info()["leaf_level"] == 3
    key = plan.export("box_key")
    level = plan.export("box_level").astype(np.int64)
    bx, by = ar.compact_bits(key), ar.compact_bits(key >> np.uint64(1))
    num = np.array([gf.paper_number(int(lv), int(a), int(b)) for lv, a, b in zip(level, bx, by)])
    assert sorted(num.tolist()) == list(range(1, 86))
    box = {int(n): i for i, n in enumerate(num)}
    child = plan.export("box_child")
    nei = plan.export("neighbor")
    inter = plan.export("interaction")
    for (kind, b), expect in gf.fig61_lists().items():
        i = box[b]
        if kind == "child":
            got = [int(num[j]) for j in child[i] if j >= 0]
        elif kind == "nei":
            got = [int(num[j]) for k, j in enumerate(nei[i]) if j >= 0 and k != 4]
        else:
            got = [int(num[j]) for j in inter[i] if j >= 0]
        assert sorted(got) == sorted(expect), (kind, b)
    plan.close()
    ctx.close()
