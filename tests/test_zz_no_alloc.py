"""GPU test of lfmm_solve_static, the solve that allocates nothing (its device buffers come
from the library's static workspace): its output equals lfmm_solve's on the same input, on
two calls in a row (the second one smaller, so that it runs over the first call's leftovers in
the workspace), and meets the FP64 oracle bar (relative l2 and max-norm <= 1e-10, eq. 1.7)."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct as od

pytestmark = pytest.mark.gpu

FMM_TOL = 1e-10


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_static_solve_equals_solve():
    import torch
    import paper_1105_3505_amd as lf
    rng = np.random.default_rng(601)
    big = wl.uniform_box(rng, 60000, 1000, origin=(-400, 77))
    fb = wl.zero_sum_loads(rng.standard_normal(len(big)))
    small = wl.uniform_box(rng, 3000, 200, origin=(5000, -20))
    fs = wl.zero_sum_loads(rng.standard_normal(len(small)))
    ctx = lf.Context(0)
    # the ordinary solves build the operators the static ones look up
    ref_big = ctx.solve(_dev(torch, big), _dev(torch, fb)).cpu().numpy()
    ref_small = ctx.solve(_dev(torch, small), _dev(torch, fs)).cpu().numpy()
    ub = torch.full((len(big),), 3.5, dtype=torch.float64, device="cuda")
    us = torch.full((len(small),), 3.5, dtype=torch.float64, device="cuda")
    xb, fbd, xs, fsd = _dev(torch, big), _dev(torch, fb), _dev(torch, small), _dev(torch, fs)
    torch.cuda.synchronize()
    ctx.solve_static(xb, fbd, ub)
    ctx.solve_static(xs, fsd, us)           # second call, smaller input
    torch.cuda.synchronize()
    u_big, u_small = ub.cpu().numpy(), us.cpu().numpy()
    assert np.array_equal(u_big, ref_big)
    assert np.array_equal(u_small, ref_small)
    for xy, f, u, seed in ((big, fb, u_big, 1), (small, fs, u_small, 2)):
        idx = wl.sample_targets(seed, len(xy), 1500)
        ref = od.direct_sum(xy[idx], xy, f)
        assert np.linalg.norm(u[idx] - ref) / np.linalg.norm(ref) <= FMM_TOL
        assert np.max(np.abs(u[idx] - ref)) / np.max(np.abs(ref)) <= FMM_TOL
    ctx.close()


def test_static_solve_limits():
    import torch
    import paper_1105_3505_amd as lf
    ctx = lf.Context(0)
    rng = np.random.default_rng(602)
    # more points than the entry point takes
    xy = wl.uniform_box(rng, 70000, 1000)
    z = torch.zeros(len(xy), dtype=torch.float64, device="cuda")
    with pytest.raises(lf.LfmmError) as e:
        ctx.solve_static(_dev(torch, xy), z, torch.empty_like(z))
    assert e.value.status == -2
    # a leaf side whose operators the context has not built yet
    xy = wl.uniform_box(rng, 2000, 300)
    f = _dev(torch, wl.zero_sum_loads(rng.standard_normal(len(xy))))
    u = torch.empty(len(xy), dtype=torch.float64, device="cuda")
    with pytest.raises(lf.LfmmError) as e:
        ctx.solve_static(_dev(torch, xy), f, u)
    assert e.value.status == -5
    # a sparse set whose deep tree exceeds the workspace: nothing computed, then a good call
    ctx.solve(_dev(torch, xy), f)
    sparse = rng.integers(-(2 ** 30), 2 ** 30, size=(60000, 2)).astype(np.int32)
    zs = torch.zeros(len(sparse), dtype=torch.float64, device="cuda")
    plan = ctx.plan(_dev(torch, sparse))          # builds its operators
    plan.close()
    with pytest.raises(lf.LfmmError) as e:
        ctx.solve_static(_dev(torch, sparse), zs, torch.empty_like(zs))
    assert e.value.status == -2
    ctx.solve_static(_dev(torch, xy), f, u)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ctx.solve(_dev(torch, xy), f).cpu().numpy())
    ctx.close()
