"""GPU tests of the C ABI's problem statement (Section 1): loads at sources, potentials wanted
at targets of the caller's choosing, zero-sum warning, invalid loads, memory footprint bound.

Parity bar: relative l2 error <= 1e-10 against the FP64 oracle's direct sum of eq. (1.7) over
the compared targets, and max |error| / max |u_ref| <= 1e-10 as well.
"""
import math
import warnings

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


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_3505_amd as lf
    c = lf.Context(0)
    yield c
    c.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(u, ref, tol=FMM_TOL):
    den2 = np.linalg.norm(ref)
    deni = np.max(np.abs(ref))
    l2 = float(np.linalg.norm(u - ref) / den2)
    mx = float(np.max(np.abs(u - ref)) / deni)
    assert l2 <= tol and mx <= tol, (l2, mx)
    return l2, mx


@pytest.mark.parametrize("case", ["disjoint", "window", "far", "coincide"])
def test_targets_distinct_from_sources(torch_mod, ctx, case):
    torch = torch_mod
    rng = np.random.default_rng(301 + ["disjoint", "window", "far", "coincide"].index(case))
    src = wl.uniform_box(rng, 20000, 700, origin=(-300, 40))
    f = wl.zero_sum_loads(rng.standard_normal(len(src)))
    if case == "disjoint":       # uniform targets in the same box, cells not holding sources
        cand = wl.uniform_box(rng, 30000, 700, origin=(-300, 40))
        have = set(map(tuple, src.tolist()))
        tgt = np.array([p for p in cand.tolist() if tuple(p) not in have][:9000], np.int32)
    elif case == "window":       # every cell of a dense window (the near field of many leaves)
        g = np.arange(100, 180)
        X, Y = np.meshgrid(g - 300, g + 40, indexing="ij")
        tgt = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.int32)
    elif case == "far":          # a few targets far outside the sources' box, plus some inside
        far = rng.integers(-10 ** 6, 10 ** 6, size=(300, 2))
        near = wl.uniform_box(rng, 300, 700, origin=(-300, 40))
        tgt = np.vstack([far, near]).astype(np.int32)
    else:                        # targets on sources (no self term), duplicated targets
        tgt = np.vstack([src[:2000], src[:500], src[:1]]).astype(np.int32)
    plan = ctx.plan(_dev(torch, src), targets=_dev(torch, tgt))
    u = plan.execute(_dev(torch, f))
    torch.cuda.synchronize()
    assert plan.info()["n_targets"] == len(tgt)
    ref = od.direct_sum(tgt, src, f)
    l2, mx = _check(u.cpu().numpy(), ref)
    print("%s: %d targets, rel l2 %.2e, max %.2e" % (case, len(tgt), l2, mx))
    # the union tree reproduces targets = sources on the shared points
    if case == "coincide":
        us = ctx.plan(_dev(torch, src)).execute(_dev(torch, f)).cpu().numpy()
        assert np.max(np.abs(u.cpu().numpy()[:2000] - us[:2000])) <= 1e-10 * np.max(np.abs(us))


def test_targets_in_a_forest(torch_mod, ctx):
    # instances with and without targets of their own share one plan; each equals a plan of
    # its own bit for bit
    torch = torch_mod
    rng = np.random.default_rng(311)
    srcs, tgts, fs = [], [], []
    for k, (n, side, m) in enumerate([(3000, 200, 1000), (50, 20, None), (8000, 900, 4000), (1, 5, 7),
                                      (2000, 60, None), (700, 5000, 300)]):
        s = wl.uniform_box(rng, n, side, origin=(int(rng.integers(-9999, 9999)), 0))
        srcs.append(s)
        fs.append(wl.zero_sum_loads(rng.standard_normal(n)) if n > 1 else np.array([1.0]))
        tgts.append(None if m is None else wl.uniform_box(rng, m, side + 10, origin=(int(s[0, 0]) - 5, -5)))
    plan = ctx.plan_batch([_dev(torch, s) for s in srcs],
                          targets=[None if t is None else _dev(torch, t) for t in tgts])
    us = plan.execute_instances([_dev(torch, f) for f in fs])
    torch.cuda.synchronize()
    for k, (s, t, f) in enumerate(zip(srcs, tgts, fs)):
        tt = s if t is None else t
        alone = ctx.plan(_dev(torch, s), targets=None if t is None else _dev(torch, t))
        ua = alone.execute(_dev(torch, f)).cpu().numpy()
        ub = us[k].cpu().numpy()
        assert ub.shape == (len(tt),)
        assert np.array_equal(ua, ub), k
        ref = od.direct_sum(tt, s, f)
        if np.max(np.abs(ref)) > 0:
            _check(ub, ref)
        alone.close()


def test_target_arguments_rejected(torch_mod, ctx):
    # through the C ABI: target coordinates with n_tgt = 0, and no target coordinates with a
    # count other than 0 or n_src, are invalid
    import ctypes
    import paper_1105_3505_amd as lf
    from paper_1105_3505_amd import _lib as L
    torch = torch_mod
    src = _dev(torch, np.zeros((4, 2), np.int32))
    tgt = _dev(torch, np.ones((3, 2), np.int32))
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    assert L._lib.lfmm_plan_create(ctx._h, 4, ctypes.c_void_p(src.data_ptr()), 0, ctypes.c_void_p(tgt.data_ptr()),
                                   st, ctypes.byref(h)) == -1
    assert L._lib.lfmm_plan_create(ctx._h, 4, ctypes.c_void_p(src.data_ptr()), 3, None, st, ctypes.byref(h)) == -1
    # targets = sources may be stated either way
    assert L._lib.lfmm_plan_create(ctx._h, 4, ctypes.c_void_p(src.data_ptr()), 4, None, st, ctypes.byref(h)) == 0
    assert L._lib.lfmm_plan_destroy(h) == 0
    with pytest.raises(ValueError):
        ctx.plan(src, targets=_dev(torch, np.zeros((0, 2), np.int32)))
    with pytest.raises(lf.LfmmError):
        # sources and targets together span 2^31 or more
        ctx.plan_batch([src], targets=[_dev(torch, np.array([[-(2 ** 31) + 5, 0], [2 ** 31 - 5, 0]], np.int32))])


def test_nonzero_total_load_warns(torch_mod, ctx):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(321)
    xy = wl.uniform_box(rng, 5000, 300)
    f = rng.uniform(0.5, 1.5, len(xy))              # total load far from zero
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        u = ctx.solve(_dev(torch, xy), _dev(torch, f))
    assert any(isinstance(x.message, lf.LfmmWarning) and x.message.status == 1 for x in w)
    _check(u.cpu().numpy(), od.direct_sum(xy, xy, f))
    # an exact zero sum gives no warning
    g = wl.zero_sum_loads(rng.standard_normal(len(xy)))
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        ctx.solve(_dev(torch, xy), _dev(torch, g))
    assert not any(isinstance(x.message, lf.LfmmWarning) for x in w)


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_non_finite_loads_rejected_before_launch(torch_mod, bad):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(331)
    xy = wl.uniform_box(rng, 4000, 250)
    f = wl.zero_sum_loads(rng.standard_normal(len(xy)))
    f[1234] = bad
    sentinel = np.full(len(xy), 7.25)
    ctx = lf.Context(0, check_loads=True)
    plan = ctx.plan(_dev(torch, xy))
    u = _dev(torch, sentinel)
    with pytest.raises(lf.LfmmError) as e:
        plan.execute(_dev(torch, f), u)
    assert e.value.status == -1
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), sentinel)        # nothing was written
    with pytest.raises(lf.LfmmError) as e:
        ctx.solve(_dev(torch, xy), _dev(torch, f), u)
    assert e.value.status == -1
    assert np.array_equal(u.cpu().numpy(), sentinel)
    # the same plan still serves good loads
    f[1234] = 0.0
    f = wl.zero_sum_loads(f)
    _check(plan.execute(_dev(torch, f)).cpu().numpy(), od.direct_sum(xy, xy, f))
    plan.close()
    ctx.close()


def _root_bits(xy):
    ext = int(max(xy[:, 0].max() - xy[:, 0].min(), xy[:, 1].max() - xy[:, 1].min())) + 1
    return max(0, math.ceil(math.log2(ext))) if ext > 1 else 0


@pytest.mark.parametrize("layout", ["uniform", "scattered", "clusters", "duplicates", "targets"])
def test_footprint_bounds_the_plan(torch_mod, ctx, layout):
    # the bytes a built plan holds never exceed lfmm_plan_footprint_bytes for its root bits,
    # whatever the layout (scattered points make deep sparse trees)
    torch = torch_mod
    rng = np.random.default_rng(341)
    tgt = None
    if layout == "uniform":
        xy = wl.uniform_box(rng, 50000, 900)
    elif layout == "scattered":
        xy = rng.integers(-(2 ** 29), 2 ** 29, size=(3000, 2)).astype(np.int32)
        xy[:70] = xy[0] + np.stack([np.arange(70) % 9, np.arange(70) // 9], axis=1)   # one full leaf
    elif layout == "clusters":
        xy = wl.gaussian_clusters(rng, 40000, rng.uniform(10 ** 4, 10 ** 6, size=(5, 2)), 300.0, 2 ** 20)
    elif layout == "duplicates":
        xy = np.repeat(wl.uniform_box(rng, 300, 40), 200, axis=0)    # 200 points per cell
    else:
        xy = wl.uniform_box(rng, 20000, 3000)
        tgt = rng.integers(-50000, 50000, size=(5000, 2)).astype(np.int32)
    allp = xy if tgt is None else np.vstack([xy, tgt])
    D = _root_bits(allp)
    plan = ctx.plan(_dev(torch, xy), targets=None if tgt is None else _dev(torch, tgt))
    info = plan.info()
    bound = ctx.footprint_bytes(len(xy), 0 if tgt is None else len(tgt), D)
    print("%s: D %d boxes %d plan bytes %d bound %d" % (layout, D, info["n_boxes"], info["device_bytes"], bound))
    assert info["root_bits"] == D
    assert 0 < info["device_bytes"] <= bound
    assert bound <= ctx.footprint_bytes(len(xy), 0 if tgt is None else len(tgt), -1)
    plan.close()
