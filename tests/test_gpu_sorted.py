"""GPU tests of lfmm_execute_sorted: loads and potentials in the plan's Morton order.

The sorted execute runs the same arithmetic as lfmm_execute, so its potentials must equal the
caller-order ones bit for bit once permuted (u_sorted[s] == u[perm[s]]); entries of points
that are not sources are never read (NaN there must not leak) and entries of points that are
not targets are never written.  One case is also checked against the FP64 oracle (direct sum
of eq. 1.7, relative l2 and max-norm <= 1e-10).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import direct as od

pytestmark = pytest.mark.gpu

SENTINEL = 12345.0


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sorted_io(plan, f, n_src, offsets=None):
    """Loads in plan order (NaN at points that are not sources) and the caller index map."""
    perm = plan.export("perm").astype(np.int64)
    n_all = len(perm)
    fs = np.full(n_all, np.nan)
    if offsets is None:
        offsets = [(0, n_all, 0, n_src)]
    for p0, p1, f0, ns in offsets:        # points [p0, p1) of an instance whose loads start at f0
        loc = perm[p0:p1]
        src = loc < ns
        fs[p0:p1][src] = f[f0 + loc[src]]
    return perm, fs


def _run_sorted(torch, plan, fs):
    u = torch.full((len(fs),), SENTINEL, dtype=torch.float64, device="cuda")
    plan.execute_sorted(_dev(torch, fs), u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("precision,adaptive,graph", [("fp64", False, False), ("mixed-bf16", False, False),
                                                      ("mixed", False, False), ("fp64", True, False),
                                                      ("fp64", False, True)])
def test_sorted_equals_caller_order(torch_mod, precision, adaptive, graph):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(1201)
    if adaptive:
        xy = wl.clusters_on_background(rng, 30000, 1 << 14)
    else:
        xy = wl.uniform_box(rng, 30000, 800)
    f = wl.zero_sum_loads(rng.standard_normal(len(xy)))
    ctx = lf.Context(0, precision=precision, adaptive=adaptive, graph=graph, max_leaf=32 if adaptive else None)
    plan = ctx.plan(_dev(torch, xy))
    u = plan.execute(_dev(torch, f)).cpu().numpy()
    perm, fs = _sorted_io(plan, f, len(xy))
    us = _run_sorted(torch, plan, fs)
    us2 = _run_sorted(torch, plan, fs)      # graph plans: recorded once, replayed
    assert np.array_equal(us, u[perm])
    assert np.array_equal(us2, us)
    if precision == "fp64" and not adaptive and not graph:
        idx = wl.sample_targets(7, len(xy), 400)
        ref = od.direct_sum(xy[idx], xy, f)
        got = u[idx]
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
    plan.close()
    ctx.close()


def test_sorted_with_separate_targets(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(1202)
    src = wl.uniform_box(rng, 15000, 600)
    tgt = wl.uniform_box(rng, 6000, 900, origin=(-150, -150))
    f = wl.zero_sum_loads(rng.standard_normal(len(src)))
    ctx = lf.Context(0)
    plan = ctx.plan(_dev(torch, src), targets=_dev(torch, tgt))
    u = plan.execute(_dev(torch, f)).cpu().numpy()
    perm, fs = _sorted_io(plan, f, len(src))
    us = _run_sorted(torch, plan, fs)
    is_tgt = perm >= len(src)
    assert is_tgt.sum() == len(tgt)
    assert np.array_equal(us[is_tgt], u[perm[is_tgt] - len(src)])
    assert np.all(us[~is_tgt] == SENTINEL)          # source-only points are not written
    plan.close()
    ctx.close()


def test_sorted_forest(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    inst = [wl.config_batched_instance(4, i) for i in range(5)]
    ctx = lf.Context(0)
    plan = ctx.plan_batch([_dev(torch, xy) for xy, _ in inst])
    us = [u.cpu().numpy() for u in plan.execute_instances([_dev(torch, f) for _, f in inst])]
    sizes = [len(xy) for xy, _ in inst]
    off = np.concatenate([[0], np.cumsum(sizes)])
    f_all = np.concatenate([f for _, f in inst])
    perm, fs = _sorted_io(plan, f_all, None,
                          offsets=[(int(off[k]), int(off[k + 1]), int(off[k]), sizes[k]) for k in range(len(inst))])
    got = _run_sorted(torch, plan, fs)
    for k in range(len(inst)):
        loc = perm[off[k]:off[k + 1]]
        assert np.array_equal(got[off[k]:off[k + 1]], us[k][loc]), k
    plan.close()
    ctx.close()
