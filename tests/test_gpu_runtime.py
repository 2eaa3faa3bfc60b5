"""GPU tests of the runtime around the passes: timing of chosen phases, plan release without a
device wait, and the sort passes that the plan build enqueues before it knows the key width.

* lfmm_plan_set_timing_phases records only the events around the chosen phases; the other
  phases come back as absent, and a mask naming no phase is rejected.
* A plan released right after its execute (no synchronisation) gives its memory back to the
  context's pool only once its stream has passed the release: plans built next, on the same
  or on another stream, must still compute exactly what a fresh context computes.
* Independent solves issued round-robin on three streams without synchronisation (the bench's
  timed loop) each equal the solve run alone, bit for bit.
* With 2^16 points or more the build sorts on two 8-bit digits before reading the root boxes
  back; when the keys are narrower than that (many points on a small box) the extra pass runs
  over zero digits and must leave the order, and so the potentials, unchanged.
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
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


def test_timing_of_chosen_phases(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(401)
    xy = wl.uniform_box(rng, 60000, 600)
    f = wl.zero_sum_loads(rng.standard_normal(60000))
    ctx = lf.Context(0)
    plan = ctx.plan(_dev(torch, xy))
    with pytest.raises(lf.LfmmError):
        plan.phase_times()                     # nothing timed yet
    from paper_1105_3505_amd import _lib as binding
    with pytest.raises(lf.LfmmError):                  # bit 6 names no phase
        binding._check(binding._lib.lfmm_plan_set_timing_phases(plan._h, 1 << 6))
    plan.set_timing_phases(["m2l", "leaf"])
    u1 = plan.execute(_dev(torch, f))
    t = plan.phase_times()
    assert set(t) == {"m2l", "leaf"} and all(v > 0 for v in t.values())
    plan.set_timing(True)
    u2 = plan.execute(_dev(torch, f))
    t_all = plan.phase_times()
    assert set(t_all) == set(plan.PHASES) and all(v >= 0 for v in t_all.values())
    plan.set_timing_phases([])                 # off: no events, the last timed execute stays
    u3 = plan.execute(_dev(torch, f))
    torch.cuda.synchronize()
    assert set(plan.phase_times()) == set(plan.PHASES)
    assert np.array_equal(u1.cpu().numpy(), u2.cpu().numpy())
    assert np.array_equal(u1.cpu().numpy(), u3.cpu().numpy())
    plan.close()
    ctx.close()


def test_release_without_wait_then_rebuild(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(402)
    sets = []
    for k in range(4):
        xy = wl.uniform_box(rng, 40000 + 5000 * k, 500 + 40 * k)
        sets.append((xy, wl.zero_sum_loads(rng.standard_normal(len(xy)))))
    # reference potentials, one fresh context per point set
    ref = []
    for xy, f in sets:
        c = lf.Context(0)
        p = c.plan(_dev(torch, xy))
        ref.append(p.execute(_dev(torch, f)).cpu().numpy())
        p.close()
        c.close()
    ctx = lf.Context(0)
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    outs = []
    for rep in range(3):
        for k, (xy, f) in enumerate(sets):
            st = s1 if (rep + k) % 2 == 0 else s2
            with torch.cuda.stream(st):
                xd, fd = _dev(torch, xy), _dev(torch, f)
                u = torch.empty(len(xy), dtype=torch.float64, device="cuda")
                plan = ctx.plan(xd, stream=st)
                plan.execute(fd, u, stream=st)
                plan.close()                   # no wait: its blocks go back after a fence
                outs.append((k, u, st))
    torch.cuda.synchronize()
    for k, u, _ in outs:
        assert np.array_equal(u.cpu().numpy(), ref[k]), "plan %d differs after pool reuse" % k
    ctx.close()


def test_extra_sort_pass_on_narrow_keys(torch_mod):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(403)
    n = 70000                                  # >= 2^16: two passes before the read-back
    xy = rng.integers(0, 16, size=(n, 2)).astype(np.int32)   # 8 key bits: one pass would do
    f = rng.standard_normal(n)
    ctx = lf.Context(0)
    plan = ctx.plan(_dev(torch, xy))
    u = plan.execute(_dev(torch, f)).cpu().numpy()
    idx = wl.sample_targets(7, n, 400)
    ref = od.direct_sum(xy[idx], xy, f)
    assert _rel(u[idx], ref) <= FMM_TOL
    pts = plan.export("points")
    assert len(pts) == n
    # Morton order inside the root box: keys never decrease along the sorted points
    def morton(p):
        x, y = int(p[0]), int(p[1])
        k = 0
        for b in range(16):
            k |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
        return k
    keys = [morton(p) for p in pts[::97]]
    assert all(a <= b for a, b in zip(keys, keys[1:]))
    plan.close()
    ctx.close()


def test_solves_in_flight_on_three_streams(torch_mod):
    """The bench's timed loop: independent solves (build, execute, release) issued round-robin
    on three streams with no synchronisation between them, each into its own output buffer,
    must each equal the solve run alone, bit for bit, for two different point sets."""
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(404)
    sets = []
    for k in range(2):
        xy = wl.uniform_box(rng, 70000 + 9000 * k, 700 + 60 * k)
        sets.append((xy, wl.zero_sum_loads(rng.standard_normal(len(xy)))))
    ctx = lf.Context(0)
    ref = []
    for xy, f in sets:
        p = ctx.plan(_dev(torch, xy))
        ref.append(p.execute(_dev(torch, f)).cpu().numpy())
        p.close()
    dev = [(_dev(torch, xy), _dev(torch, f)) for xy, f in sets]
    streams = [torch.cuda.current_stream(), torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for i in range(12):
        k = (i // 3) % 2
        st = streams[i % 3]
        xd, fd = dev[k]
        u = torch.empty(len(sets[k][0]), dtype=torch.float64, device="cuda")
        with torch.cuda.stream(st):
            plan = ctx.plan(xd, stream=st)
            plan.execute(fd, u, stream=st)
            plan.close()
        outs.append((k, u))
    torch.cuda.synchronize()
    for k, u in outs:
        assert np.array_equal(u.cpu().numpy(), ref[k])
    idx = wl.sample_targets(9, len(sets[0][0]), 300)
    assert _rel(ref[0][idx], od.direct_sum(sets[0][0][idx], sets[0][0], sets[0][1])) <= FMM_TOL
    ctx.close()
