"""GPU tests of HIP-graph replay of the evaluation passes and of the N_leaf autotuner.

A graph replays the same kernels with the same arguments, so its potentials must equal the
eagerly launched ones bit for bit, for every replay and for new load/potential buffers.  The
autotuner must return one of its candidates, and a context in automatic mode must then build
the same tree as one given that N_leaf explicitly.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import direct as od

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed-bf16"])
def test_graph_replay_equals_eager(torch_mod, precision):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(301)
    xy = wl.uniform_box(rng, 30000, 800)
    loads = [wl.zero_sum_loads(rng.standard_normal(30000)) for _ in range(3)]
    eager = lf.Context(0, precision=precision)
    graph = lf.Context(0, precision=precision, graph=True)
    pe, pg = eager.plan(_dev(torch, xy)), graph.plan(_dev(torch, xy))
    for f in loads:
        fd = _dev(torch, f)
        ue = pe.execute(fd)
        ug = pg.execute(fd)          # first call records the graph, later calls replay it
        ug2 = pg.execute(fd)
        torch.cuda.synchronize()
        assert np.array_equal(ue.cpu().numpy(), ug.cpu().numpy())
        assert np.array_equal(ue.cpu().numpy(), ug2.cpu().numpy())
    idx = wl.sample_targets(5, 30000, 300)
    tol = 1e-10 if precision == "fp64" else 1e-7
    ref = od.direct_sum(xy[idx], xy, loads[-1])
    assert np.linalg.norm(ug2.cpu().numpy()[idx] - ref) <= tol * np.linalg.norm(ref)
    pe.close(); pg.close(); eager.close(); graph.close()


def test_graph_replay_batched(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    inst = [wl.config_batched_instance(4, i) for i in range(24)]
    eager = lf.Context(0)
    graph = lf.Context(0, graph=True)
    pe = eager.plan_batch([_dev(torch, xy) for xy, _ in inst])
    pg = graph.plan_batch([_dev(torch, xy) for xy, _ in inst])
    fs = [_dev(torch, f) for _, f in inst]
    ue = pe.execute_instances(fs)
    ug = pg.execute_instances(fs)
    ug = pg.execute_instances([f * 2.0 for f in fs])   # new buffers through the pointer table
    torch.cuda.synchronize()
    for a, b in zip(ue, ug):
        assert np.array_equal(2.0 * a.cpu().numpy(), b.cpu().numpy())
    pe.close(); pg.close(); eager.close(); graph.close()


def test_autotune_choice_is_used_in_auto_mode(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(303)
    xy = _dev(torch, wl.uniform_box(rng, 200000, 1800))
    ctx = lf.Context(0, max_leaf=0)
    best, times = ctx.autotune(xy, candidates=(16, 32, 64, 128), objective="execute", reps=2)
    assert best in (16, 32, 64, 128) and all(t > 0 for t in times.values())
    assert times[best] == min(times.values())
    auto = ctx.plan(xy).info()
    fixed_ctx = lf.Context(0, max_leaf=best)
    fixed = fixed_ctx.plan(xy).info()
    assert (auto["leaf_level"], auto["n_leaves"]) == (fixed["leaf_level"], fixed["n_leaves"])
    ctx.close(); fixed_ctx.close()


def test_autotuned_forest_takes_each_class_choice(torch_mod):
    # instances of two size classes tuned separately; a forest in automatic mode gives each
    # instance its class's N_leaf, so each equals its own plan built with that value bit for bit
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(304)
    small = wl.uniform_box(rng, 3000, int(4 * 3000 ** 0.5))
    large = wl.uniform_box(rng, 60000, int(4 * 60000 ** 0.5))
    fa = wl.zero_sum_loads(rng.standard_normal(len(small)))
    fb = wl.zero_sum_loads(rng.standard_normal(len(large)))
    ctx = lf.Context(0, max_leaf=0)
    best = {}
    for name, xy in (("small", small), ("large", large)):
        best[name], times = ctx.autotune(_dev(torch, xy), candidates=(8, 32, 128), objective="execute", reps=2)
        assert times[best[name]] == min(times.values())
    for order in (("small", "large"), ("large", "small")):
        pts = {"small": (small, fa), "large": (large, fb)}
        forest = ctx.plan_batch([_dev(torch, pts[k][0]) for k in order])
        us = forest.execute_instances([_dev(torch, pts[k][1]) for k in order])
        for k, u in zip(order, us):
            own_ctx = lf.Context(0, max_leaf=best[k])
            own = own_ctx.plan(_dev(torch, pts[k][0]))
            ref = own.execute(_dev(torch, pts[k][1]))
            torch.cuda.synchronize()
            assert np.array_equal(u.cpu().numpy(), ref.cpu().numpy()), (order, k)
            own.close()
            own_ctx.close()
        forest.close()
    ctx.close()


def test_autotune_batch_whole_forest(torch_mod):
    # one N_leaf timed on the whole forest, then used for every instance in automatic mode
    import paper_1105_3505_amd as lf
    torch = torch_mod
    inst = [wl.config_batched_instance(4, i) for i in range(12)]
    xs = [_dev(torch, xy) for xy, _ in inst]
    ctx = lf.Context(0, max_leaf=0)
    best, times = ctx.autotune_batch(xs, candidates=(16, 64, 128), objective="execute", reps=2)
    assert best in (16, 64, 128) and times[best] == min(times.values())
    forest = ctx.plan_batch(xs)
    us = forest.execute_instances([_dev(torch, f) for _, f in inst])
    fixed_ctx = lf.Context(0, max_leaf=best)
    fixed = fixed_ctx.plan_batch(xs)
    ref = fixed.execute_instances([_dev(torch, f) for _, f in inst])
    torch.cuda.synchronize()
    for a, b in zip(us, ref):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    forest.close(); fixed.close(); ctx.close(); fixed_ctx.close()
