"""Out-of-memory paths, forced from the host: with LFMM_TEST_FAIL_ALLOC=k the k-th device block
requested after the variable is set fails as a failed hipMalloc would.  Every failure must
surface as LFMM_E_NOMEM from the call that needed the block (context creation, plan build,
adaptive list build), leave nothing behind that later calls trip over, and a complete solve
right after must give the same potentials, bit for bit, as one that never saw a failure."""
import os

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

NOMEM = -3


def _solve(torch, lf, xy, f, **opts):
    ctx = lf.Context(0, **opts)
    try:
        plan = ctx.plan(torch.from_numpy(xy).cuda())
        u = plan.execute(torch.from_numpy(f).cuda())
        torch.cuda.synchronize()
        out = u.cpu().numpy()
        plan.close()
        return out
    finally:
        ctx.close()


@pytest.mark.parametrize("opts", [{}, {"adaptive": True, "max_leaf": 16}])
def test_injected_allocation_failures(opts):
    import torch
    import paper_1105_3505_amd as lf
    xy = wl.clusters_on_background(np.random.default_rng(3), 6000, 1 << 14)
    f = wl.zero_sum_loads(np.random.default_rng(4).standard_normal(len(xy)))
    ref = _solve(torch, lf, xy, f, **opts)
    failures = 0
    for k in range(1, 16):
        os.environ["LFMM_TEST_FAIL_ALLOC"] = str(k)
        try:
            _solve(torch, lf, xy, f, **opts)
        except lf.LfmmError as e:
            assert e.status == NOMEM, (k, e)
            failures += 1
        finally:
            del os.environ["LFMM_TEST_FAIL_ALLOC"]
        assert np.array_equal(_solve(torch, lf, xy, f, **opts), ref), k
    print("forced failures:", failures)
    assert failures >= 4
