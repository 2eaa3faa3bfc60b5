"""GPU parity on the measurement configurations at their full sizes, against the FP64 oracle
(direct sum of eq. 1.7) on sampled targets:

* 2,000,000 sources in 64 Gaussian clusters over a 2^20 x 2^20 region, mixed precision
  (FP32 hi/lo or three-part bf16 matrix-core M2L), tolerance 1e-7;
* the 512-instance batch (sizes log-uniform in [1e3, 1e5]) as one forest plan, FP64
  (tolerance 1e-10) and both mixed forms (1e-7);
* serving requests up to ~8.7e5 points through the continuous-batching server.

Each check asserts the relative l2 error and the max-norm error max |u - u_ref| / max |u_ref|.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import direct as od

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = {"fp64": 1e-10, "mixed": 1e-7, "mixed-bf16": 1e-7}


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _errs(u, ref):
    return (float(np.linalg.norm(u - ref) / np.linalg.norm(ref)),
            float(np.max(np.abs(u - ref)) / np.max(np.abs(ref))))


@pytest.mark.parametrize("precision", ["mixed", "mixed-bf16"])
def test_clusters_mixed_full_size(torch_mod, precision):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    xy, f = wl.config_clusters()
    ctx = lf.Context(0, precision=precision)
    plan = ctx.plan(_dev(torch, xy))
    u = plan.execute(_dev(torch, f))
    torch.cuda.synchronize()
    idx = wl.sample_targets(22, len(xy), 1000)
    ref = od.direct_sum(xy[idx], xy, f)
    l2, mx = _errs(u.cpu().numpy()[idx], ref)
    info = plan.info()
    print("2e6 clusters %s: leaf side %d, %d boxes, rel l2 %.3e, max %.3e"
          % (precision, info["leaf_side"], info["n_boxes"], l2, mx))
    assert l2 <= TOL[precision] and mx <= TOL[precision]
    plan.close()
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed-bf16"])
def test_batched_512_full_forest(torch_mod, precision):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    inst = wl.config_batched()
    assert len(inst) == 512
    ctx = lf.Context(0, precision=precision)
    plan = ctx.plan_batch([_dev(torch, xy) for xy, _ in inst])
    us = plan.execute_instances([_dev(torch, f) for _, f in inst])
    torch.cuda.synchronize()
    worst_l2 = worst_mx = 0.0
    num = den = 0.0
    for k, (xy, f) in enumerate(inst):
        idx = wl.sample_targets(40 + k, len(xy), 40)
        ref = od.direct_sum(xy[idx], xy, f)
        uk = us[k].cpu().numpy()[idx]
        l2, mx = _errs(uk, ref)
        worst_l2, worst_mx = max(worst_l2, l2), max(worst_mx, mx)
        num += float(np.sum((uk - ref) ** 2))
        den += float(np.sum(ref ** 2))
    pooled = (num / den) ** 0.5
    print("512 instances %s: pooled rel l2 %.3e, worst instance l2 %.3e, worst max %.3e"
          % (precision, pooled, worst_l2, worst_mx))
    assert pooled <= TOL[precision]
    assert worst_l2 <= TOL[precision] and worst_mx <= TOL[precision]
    plan.close()
    ctx.close()


def test_serving_large_requests(torch_mod):
    # requests 8 (874,945 points) and 118 (708,383) of the serving stream with small ones
    # around them, all in flight together; each equals its solve alone bit for bit and meets
    # the oracle bar on sampled targets
    import paper_1105_3505_amd as lf
    torch = torch_mod
    picks = [8, 0, 1, 118, 2, 3, 4]
    reqs = [wl.config_serving_request(5, i)[:2] for i in picks]
    dev = [(_dev(torch, xy), _dev(torch, f)) for xy, f in reqs]
    ctx = lf.Context(0)
    srv = lf.Server(ctx, max_batch=4, max_inflight=3)
    tickets = [srv.submit(*d) for d in dev]
    out = [srv.wait(t, timeout=300) for t in tickets]
    srv.close()
    alone = lf.Context(0)
    for (xy, f), (u, st), d, i in zip(reqs, out, dev, picks):
        assert st["status"] == 0
        ua = alone.solve(*d).cpu().numpy()
        assert np.array_equal(u.cpu().numpy(), ua), i
        idx = wl.sample_targets(500 + i, len(xy), 400)
        l2, mx = _errs(u.cpu().numpy()[idx], od.direct_sum(xy[idx], xy, f))
        print("request %d (n=%d, batch of %d): rel l2 %.3e max %.3e" % (i, len(xy), st["batch_size"], l2, mx))
        assert l2 <= TOL["fp64"] and mx <= TOL["fp64"]
    alone.close()
    ctx.close()
