"""GPU pass-by-pass checks: each kernel against a host FP64 product of the same operators.

The tree (Section 6, Definition 6.1) is rebuilt by brute force from the exported Morton
order; P2M, M2M, M2L and L2L (Section 8.2 steps 1-4) are recomputed on the host from the
exported expansions and the host copy of the operators, so a kernel bug shows up in the
pass where it happens rather than only in the final potential.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

RANK = 48


def _spread(v):
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for b in range(32):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
    return out


def _morton(x, y):
    return _spread(x) | (_spread(y) << np.uint64(1))


def _slots(c):
    cx, cy = c & 1, c >> 1
    out = []
    for dy in range(-2 - cy, 4 - cy):
        for dx in range(-2 - cx, 4 - cx):
            if abs(dx) <= 1 and abs(dy) <= 1:
                continue
            out.append((dx, dy))
    return out


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_1105_3505_amd as lf
    ctx = lf.Context(0)
    yield torch, lf, ctx
    ctx.close()


def _run(setup, xy, f):
    torch, lf, ctx = setup
    plan = ctx.plan(torch.from_numpy(xy).cuda())
    u = plan.execute(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ex = {k: plan.export(k) for k in lf.Plan.EXPORTS}
    return plan, u.cpu().numpy(), ex, plan.info()


CASES = {
    "small_uniform": lambda: wl.config_small_uniform(),
    "uniform_20k": lambda: (lambda r: (wl.uniform_box(r, 20000, 700), wl.zero_sum_loads(r.standard_normal(20000))))(
        np.random.default_rng(31)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_tree_matches_brute_force(setup, case):
    xy, f = CASES[case]()
    plan, _, ex, info = _run(setup, xy, f)
    D, L = info["root_bits"], info["leaf_level"]
    pts, perm = ex["points"], ex["perm"]
    lo = xy.min(axis=0)
    assert np.array_equal(np.sort(perm), np.arange(len(xy)))
    assert np.array_equal(pts, (xy[perm] - lo).astype(np.int32))
    keys = _morton(pts[:, 0], pts[:, 1])
    assert np.all(keys[1:] >= keys[:-1])
    base, count = ex["level_base"], ex["level_count"]
    assert len(base) == L + 1 and len(count) == L + 1
    # boxes are numbered by height above the leaves: leaves first, the root last
    assert base[L] == 0 and base[0] == info["n_boxes"] - 1 and count[0] == 1
    off = {lev: (int(base[lev]), int(base[lev] + count[lev])) for lev in range(L + 1)}
    assert np.array_equal(ex["box_level"][off[L][0]:off[L][1]], np.full(count[L], L, np.int8))
    bkey, b0, b1 = ex["box_key"], ex["box_begin"], ex["box_end"]
    for lev in range(L + 1):
        pk = keys >> np.uint64(2 * (D - lev))
        uk, first = np.unique(pk, return_index=True)
        sl = slice(*off[lev])
        assert np.array_equal(bkey[sl], uk), lev
        assert np.array_equal(b0[sl], first), lev
        assert np.array_equal(b1[sl], np.append(first[1:], len(pts))), lev
    # leaf occupancy rule of Section 6
    leaves = slice(*off[L])
    assert np.max(b1[leaves] - b0[leaves]) <= 64 or L == D
    index = [{int(k): off[lev][0] + i for i, k in enumerate(bkey[slice(*off[lev])])} for lev in range(L + 1)]
    par, ch = ex["box_parent"], ex["box_child"]
    for lev in range(L + 1):
        for g in range(*off[lev]):
            k = int(bkey[g])
            assert par[g] == (index[lev - 1][k >> 2] if lev else -1)
            for c in range(4):
                want = index[lev + 1].get(4 * k + c, -1) if lev < L else -1
                assert ch[g, c] == want
    il = ex["interaction"]
    for lev in range(2):
        assert np.all(il[slice(*off[lev])] == -1)
    for lev in range(2, L + 1):
        for g in range(*off[lev]):
            k = int(bkey[g])
            bx = int(_compact(k))
            by = int(_compact(k >> 1))
            c = (bx & 1) + 2 * (by & 1)
            for s, (dx, dy) in enumerate(_slots(c)):
                x, y = bx + dx, by + dy
                want = -1
                if 0 <= x < 2 ** lev and 0 <= y < 2 ** lev:
                    want = index[lev].get(int(_morton(np.array([x]), np.array([y]))[0]), -1)
                assert il[g, s] == want
    nl = ex["neighbor"]
    for lev in range(L + 1):
        for g in range(*off[lev]):
            k = int(bkey[g])
            bx, by = int(_compact(k)), int(_compact(k >> 1))
            q = 0
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    x, y = bx + dx, by + dy
                    want = -1
                    if 0 <= x < 2 ** lev and 0 <= y < 2 ** lev:
                        want = index[lev].get(int(_morton(np.array([x]), np.array([y]))[0]), -1)
                    assert nl[g, q] == want
                    q += 1


def _compact(k):
    k = int(k)
    out = 0
    for b in range(32):
        out |= ((k >> (2 * b)) & 1) << b
    return out


@pytest.mark.parametrize("case", sorted(CASES))
def test_passes_match_host_products(setup, case):
    torch, lf, ctx = setup
    xy, f = CASES[case]()
    plan, u, ex, info = _run(setup, xy, f)
    D, L, side = info["root_bits"], info["leaf_level"], info["leaf_side"]
    assert L >= 2
    ops = lf.HostOperators(side, L - 1)
    ranks = [ops.level(h)[1] for h in range(L - 1)]
    base, count = ex["level_base"], ex["level_count"]
    off = {lev: (int(base[lev]), int(base[lev] + count[lev])) for lev in range(L + 1)}
    bkey, b0, b1 = ex["box_key"], ex["box_begin"], ex["box_end"]
    pts, fs, Q, U = ex["points"], ex["loads"], ex["qhat"], ex["uhat"]
    perm = ex["perm"]
    assert np.array_equal(fs, f[perm])
    # padded slots stay zero
    for lev in range(2, L + 1):
        r = ranks[L - lev]
        assert not np.any(Q[slice(*off[lev]), r:]) and not np.any(U[slice(*off[lev]), r:])

    def close(a, b, what):
        scale = max(np.max(np.abs(b)), 1e-300)
        err = np.max(np.abs(a - b)) / scale
        assert err <= 1e-12, "%s: %.3e" % (what, err)

    # P2M
    T = ops.leaf()
    r0 = ranks[0]
    ref = np.zeros((count[L], r0))
    for i, g in enumerate(range(*off[L])):
        k = int(bkey[g])
        cx, cy = _compact(k) * side, _compact(k >> 1) * side
        p = pts[b0[g]:b1[g]]
        loc = (p[:, 0] - cx) + side * (p[:, 1] - cy)
        ref[i] = T[:, loc] @ fs[b0[g]:b1[g]]
    close(Q[slice(*off[L]), :r0], ref, "P2M")
    # M2M
    ch = ex["box_child"]
    for lev in range(L - 1, 1, -1):
        h = L - lev
        ref = np.zeros((count[lev], ranks[h]))
        for i, g in enumerate(range(*off[lev])):
            for c in range(4):
                if ch[g, c] >= 0:
                    ref[i] += ops.ofo(h, c) @ Q[ch[g, c], :ranks[h - 1]]
        close(Q[slice(*off[lev]), :ranks[h]], ref, "M2M level %d" % lev)
    # M2L (+ L2L below level 2)
    il, par = ex["interaction"], ex["box_parent"]
    for lev in range(2, L + 1):
        h = L - lev
        sk = ops.skeleton(h)
        s_h = side << h
        Tcache = {}
        ref = np.zeros((count[lev], ranks[h]))
        for i, g in enumerate(range(*off[lev])):
            k = int(bkey[g])
            c = (_compact(k) & 1) + 2 * (_compact(k >> 1) & 1)
            for s, d in enumerate(_slots(c)):
                src = il[g, s]
                if src < 0:
                    continue
                if d not in Tcache:
                    diff = sk[:, None, :] - sk[None, :, :] - np.array(d) * s_h
                    Tcache[d] = lf.host_phi(diff.reshape(-1, 2)).reshape(len(sk), len(sk))
                ref[i] += Tcache[d] @ Q[src, :ranks[h]]
            if lev >= 3:
                ref[i] += ops.ofo(h + 1, int(k & 3)).T @ U[par[g], :ranks[h + 1]]
        close(U[slice(*off[lev]), :ranks[h]], ref, "M2L+L2L level %d" % lev)
