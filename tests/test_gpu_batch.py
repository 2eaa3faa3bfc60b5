"""GPU parity of forest plans: many independent point sets in one plan (shared launches).

Every instance of a forest plan has its own root box and tree, built exactly as a plan of its
own would build it, and every pass computes a box's result from that box's own operands in a
fixed order.  So the potentials of an instance evaluated in a batch must equal, bit for bit,
those of the same instance evaluated alone; both must also meet the FP64 accuracy target
against the oracle (relative l2 <= 1e-10, eq. 1.7).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import direct as od

pytestmark = pytest.mark.gpu

FMM_TOL = 1e-10


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(u, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(u - ref) / (den if den > 0 else 1.0))


def _mixed_instances(seed):
    """Sizes and extents chosen so that the forest holds trees of leaf level 0, 1 and >= 2,
    several leaf sides, duplicates and single points."""
    rng = np.random.default_rng(seed)
    out = []
    for n, side in [(1, 8), (2, 3), (40, 30), (65, 64), (300, 90), (2500, 2500), (5000, 300),
                    (800, 10000), (3000, 181), (12000, 640)]:
        xy = wl.uniform_box(rng, n, side, origin=(int(rng.integers(-10 ** 6, 10 ** 6)),
                                                  int(rng.integers(-10 ** 6, 10 ** 6))))
        f = wl.zero_sum_loads(rng.standard_normal(n)) if n > 1 else np.array([0.75])
        out.append((xy, f))
    base = wl.uniform_box(rng, 400, 50)
    xy = np.vstack([base, base[:100]])            # duplicate points
    out.append((xy, rng.standard_normal(len(xy))))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(torch_mod, precision):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    ctx = lf.Context(0, precision=precision)
    inst = _mixed_instances(71)
    plan = ctx.plan_batch([_dev(torch, xy) for xy, _ in inst])
    us = plan.execute_instances([_dev(torch, f) for _, f in inst])
    torch.cuda.synchronize()
    info = plan.info()
    assert info["n_instances"] == len(inst) and info["n_points"] == sum(len(f) for _, f in inst)
    tol = FMM_TOL if precision == "fp64" else 1e-7
    for k, (xy, f) in enumerate(inst):
        alone = ctx.plan(_dev(torch, xy))
        ua = alone.execute(_dev(torch, f)).cpu().numpy()
        ub = us[k].cpu().numpy()
        assert np.array_equal(ua, ub), "instance %d differs from its own plan" % k
        if len(f) > 1:
            assert _rel(ub, od.direct_sum(xy, xy, f)) <= tol, k
        else:
            assert ub[0] == 0.0
        alone.close()
    # a second execute with other loads reuses the plan
    gs = [np.asarray(f)[::-1].copy() for _, f in inst]
    us2 = plan.execute_instances([_dev(torch, g) for g in gs])
    torch.cuda.synchronize()
    for k in (3, 6, 9):
        xy = inst[k][0]
        assert _rel(us2[k].cpu().numpy(), od.direct_sum(xy, xy, gs[k])) <= tol
    plan.close()
    ctx.close()


def test_batch_tree_exports(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    ctx = lf.Context(0)
    inst = _mixed_instances(72)[:8]
    plan = ctx.plan_batch([_dev(torch, xy) for xy, _ in inst])
    bi, bl = plan.export("box_instance"), plan.export("box_level")
    par, b0, b1 = plan.export("box_parent"), plan.export("box_begin"), plan.export("box_end")
    perm = plan.export("perm")
    sizes = [len(f) for _, f in inst]
    off = np.concatenate([[0], np.cumsum(sizes)])
    # points of instance k are [off[k], off[k+1]) and its perm is a permutation of its indices
    for k in range(len(inst)):
        assert np.array_equal(np.sort(perm[off[k]:off[k + 1]]), np.arange(sizes[k]))
    # one root per instance; every box inside its instance's point range; parent one level up
    roots = np.flatnonzero(par < 0)
    assert sorted(bi[roots]) == list(range(len(inst)))
    assert np.all(b0 >= off[bi]) and np.all(b1 <= off[bi + 1]) and np.all(b1 > b0)
    child = par >= 0
    assert np.all(bi[par[child]] == bi[child]) and np.all(bl[par[child]] == bl[child] - 1)
    plan.close()
    ctx.close()


def test_batched_workload_sample(torch_mod):
    # 64 instances of the batched workload recipe (log-uniform sizes 1e3 .. 1e5)
    import paper_1105_3505_amd as lf
    torch = torch_mod
    ctx = lf.Context(0)
    inst = [wl.config_batched_instance(4, i) for i in range(64)]
    plan = ctx.plan_batch([_dev(torch, xy) for xy, _ in inst])
    us = plan.execute_instances([_dev(torch, f) for _, f in inst])
    torch.cuda.synchronize()
    for k in range(0, 64, 9):
        xy, f = inst[k]
        idx = wl.sample_targets(100 + k, len(xy), 300)
        assert _rel(us[k].cpu().numpy()[idx], od.direct_sum(xy[idx], xy, f)) <= FMM_TOL, k
    plan.close()
    ctx.close()


def test_batch_rejects_bad_input(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    ctx = lf.Context(0)
    good = _dev(torch, np.zeros((3, 2), np.int32))
    empty = _dev(torch, np.zeros((0, 2), np.int32))
    with pytest.raises(lf.LfmmError) as e:
        ctx.plan_batch([good, empty])
    assert e.value.status == -1
    far = _dev(torch, np.array([[-(2 ** 31) + 5, 0], [2 ** 31 - 5, 0]], np.int32))
    with pytest.raises(lf.LfmmError) as e:
        ctx.plan_batch([good, far])
    assert e.value.status == -2
    ctx.close()


def test_large_instances_in_one_forest(torch_mod):
    """Instances of a few hundred thousand points each: the plan build counts each instance's
    level statistics over many chunks (into several copies of the counters), for every
    instance of the forest at once; each instance must still get the tree, and the bits, of
    its own plan, and meet the FP64 target on sampled targets."""
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(1301)
    inst = []
    for n, side, origin in [(300000, 2500, (0, 0)), (280000, 600, (10 ** 6, -(10 ** 6))),
                            (3000, 100, (-5000, 70))]:
        xy = wl.uniform_box(rng, n, side, origin=origin)
        inst.append((xy, wl.zero_sum_loads(rng.standard_normal(n))))
    ctx = lf.Context(0)
    plan = ctx.plan_batch([_dev(torch, xy) for xy, _ in inst])
    us = plan.execute_instances([_dev(torch, f) for _, f in inst])
    torch.cuda.synchronize()
    for k, (xy, f) in enumerate(inst):
        alone = ctx.plan(_dev(torch, xy))
        ua = alone.execute(_dev(torch, f)).cpu().numpy()
        ub = us[k].cpu().numpy()
        assert np.array_equal(ua, ub), "instance %d differs from its own plan" % k
        idx = wl.sample_targets(11 + k, len(xy), 300)
        ref = od.direct_sum(xy[idx], xy, f)
        assert _rel(ub[idx], ref) <= FMM_TOL, k
        assert np.max(np.abs(ub[idx] - ref)) <= FMM_TOL * np.max(np.abs(ref)), k
        alone.close()
    plan.close()
    ctx.close()
