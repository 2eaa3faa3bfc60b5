"""GPU checks of the adaptive tree (LFMM_FLAG_ADAPTIVE; Section 6, closing paragraph).

* Roles and the U, V, W, X lists the library builds (small boxes taking the direct route)
  equal, box for box, those of the brute-force reference (tests/adaptive_ref.py, pinned on the
  CPU), and count every (target leaf, source leaf) pair exactly once.
* Potentials against the FP64 oracle (eq. 1.7): relative l2 and max-norm errors <= 1e-10 in
  FP64, <= 1e-7 with the mixed-precision M2L, on point sets whose leaves spread over many
  levels (dense clusters on a sparse background, whose widest leaves exceed the device phi
  table), with separate targets, the 9-point operator, batches, graph replay and degenerate
  sizes.
"""
import numpy as np
import pytest

import adaptive_ref as ar
import workloads as wl
from oracle import direct as od

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-7
DIRECT_MAX = 48   # boxes with at most this many points take no expansion route (the skeleton size)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def lf():
    import paper_1105_3505_amd as m
    return m


_CTX = {}


def _ctx(lf, **opts):
    key = tuple(sorted(opts.items()))
    if key not in _CTX:
        _CTX[key] = lf.Context(0, adaptive=True, **opts)
    return _CTX[key]


def teardown_module(module):
    for c in _CTX.values():
        c.close()
    _CTX.clear()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(u, ref):
    return float(np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-300))


def _maxrel(u, ref):
    return float(np.max(np.abs(u - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _loads(seed, n):
    return wl.zero_sum_loads(np.random.default_rng(seed).uniform(-1.0, 1.0, n))


def _solve(torch, ctx, xy, f, targets=None):
    plan = ctx.plan(_dev(torch, xy), targets=None if targets is None else _dev(torch, targets))
    u = plan.execute(_dev(torch, f))
    torch.cuda.synchronize()
    return u.cpu().numpy(), plan


def _check(u, ref, tol, label):
    e2, em = _rel(u, ref), _maxrel(u, ref)
    print("%s: rel l2 %.3e, rel max %.3e" % (label, e2, em))
    assert e2 <= tol and em <= tol


# ---- lists ---------------------------------------------------------------------------------

LIST_CASES = {
    "background_3k": (lambda: wl.clusters_on_background(np.random.default_rng(11), 3000, 1 << 14), 16),
    "clusters_4k": (lambda: wl.gaussian_clusters(np.random.default_rng(12), 4000,
                                                 np.array([[900.0, 700.0], [2600.0, 3100.0]]), 120.0, 4096), 8),
    "background_2k_wide": (lambda: wl.clusters_on_background(np.random.default_rng(13), 2000, 1 << 20,
                                                             background=0.5), 32),
}


@pytest.mark.parametrize("case", sorted(LIST_CASES))
def test_lists_match_reference(torch_mod, lf, case):
    make, max_leaf = LIST_CASES[case]
    xy = make()
    ctx = _ctx(lf, max_leaf=max_leaf)
    plan = ctx.plan(_dev(torch_mod, xy))
    info = plan.info()
    assert info["adaptive"] == 1
    key = plan.export("box_key")
    level = plan.export("box_level").astype(np.int64)
    parent = plan.export("box_parent")
    count = (plan.export("box_end") - plan.export("box_begin")).astype(np.int64)
    inst = plan.export("box_instance")
    bx, by = ar.compact_bits(key), ar.compact_bits(key >> np.uint64(1))
    role = plan.export("box_role")
    ref_role = ar.roles(level, parent, count, max_leaf, info["leaf_level"])
    assert np.array_equal(role, ref_role)
    U, V, W, X = ar.lists(level, bx, by, parent, inst, ref_role, count, DIRECT_MAX)
    got = {}
    for name in "UWX":
        off, ent = plan.export_list(name)
        got[name] = [sorted(ent[off[b]:off[b + 1]].tolist()) for b in range(len(level))]
    il = plan.export("interaction")
    got["V"] = [sorted(int(v) for v in il[b] if v >= 0) for b in range(len(level))]
    for name, ref in zip("UVWX", (U, V, W, X)):
        bad = [b for b in range(len(level)) if got[name][b] != ref[b]]
        assert not bad, "%s list differs at boxes %s" % (name, bad[:5])
    leaf_levels = sorted(set(level[role == ar.LEAF].tolist()))
    _, _, Wb, Xb = ar.lists(level, bx, by, parent, inst, ref_role)   # before the direct rule
    print("%s: %d boxes, leaves on levels %s, |W| %d (%d before the direct rule), |X| %d (%d)" % (
        case, len(level), leaf_levels, sum(map(len, W)), sum(map(len, Wb)), sum(map(len, X)), sum(map(len, Xb))))
    assert len(leaf_levels) >= 3 and sum(map(len, Wb)) > 0 and sum(map(len, Xb)) > 0
    cov = ar.coverage(parent, role, got["U"], got["V"], got["W"], got["X"], inst)
    assert set(cov.values()) == {1}
    plan.close()


# ---- potentials ----------------------------------------------------------------------------

PARITY_CASES = {
    # name: (points, max_leaf)
    "background_20k": (lambda: wl.clusters_on_background(np.random.default_rng(21), 20000, 1 << 16), 32),
    "background_12k_wide": (lambda: wl.clusters_on_background(np.random.default_rng(22), 12000, 1 << 22,
                                                              background=0.4), 24),
    "clusters_30k": (lambda: wl.gaussian_clusters(np.random.default_rng(23), 30000,
                                                  np.array([[3000.0, 2000.0], [9000.0, 11000.0],
                                                            [12000.0, 3000.0]]), 400.0, 16384), 16),
    "uniform_20k": (lambda: wl.uniform_box(np.random.default_rng(24), 20000, 700), 64),
}


@pytest.mark.parametrize("case", sorted(PARITY_CASES))
def test_parity_fp64(torch_mod, lf, case):
    make, max_leaf = PARITY_CASES[case]
    xy = make()
    f = _loads(7, len(xy))
    u, plan = _solve(torch_mod, _ctx(lf, max_leaf=max_leaf), xy, f)
    info = plan.info()
    print(case, {k: info[k] for k in ("leaf_level", "n_boxes", "n_leaves", "near_pairs", "m2l_pairs",
                                      "m2p_terms", "p2l_terms")})
    if case != "uniform_20k":
        assert info["m2p_terms"] > 0 and info["p2l_terms"] > 0
    _check(u, od.direct_sum(xy, xy, f), FP64_TOL, case)
    plan.close()


@pytest.mark.parametrize("precision", ["mixed", "mixed-bf16"])
@pytest.mark.parametrize("case", ["background_20k", "clusters_30k"])
def test_parity_mixed(torch_mod, lf, case, precision):
    make, max_leaf = PARITY_CASES[case]
    xy = make()
    f = _loads(8, len(xy))
    u, plan = _solve(torch_mod, _ctx(lf, max_leaf=max_leaf, precision=precision), xy, f)
    _check(u, od.direct_sum(xy, xy, f), MIXED_TOL, case + " " + precision)
    plan.close()


def test_separate_targets(torch_mod, lf):
    rng = np.random.default_rng(31)
    xy = wl.clusters_on_background(rng, 15000, 1 << 15)
    tg = wl.clusters_on_background(np.random.default_rng(32), 5000, 1 << 15)
    f = _loads(9, len(xy))
    u, plan = _solve(torch_mod, _ctx(lf, max_leaf=32), xy, f, targets=tg)
    assert u.shape == (len(tg),)
    _check(u, od.direct_sum(tg, xy, f), FP64_TOL, "targets")
    plan.close()


def test_nine_point_operator(torch_mod, lf):
    # inside a 128 x 128 square: the oracle tabulates the 9-point phi to radius 128
    xy = wl.clusters_on_background(np.random.default_rng(41), 3000, 128, sigma=10.0)
    f = _loads(10, len(xy))
    u, plan = _solve(torch_mod, _ctx(lf, max_leaf=16, stencil=9), xy, f)
    _check(u, od.direct_sum(xy, xy, f, stencil=9), FP64_TOL, "9-point")
    plan.close()


def test_batch_of_instances(torch_mod, lf):
    torch = torch_mod
    xys = [wl.clusters_on_background(np.random.default_rng(50 + k), n, ext)
           for k, (n, ext) in enumerate([(6000, 1 << 14), (3000, 1 << 18), (9000, 1 << 12)])]
    fs = [_loads(60 + k, len(x)) for k, x in enumerate(xys)]
    plan = _ctx(lf, max_leaf=32).plan_batch([_dev(torch, x) for x in xys])
    us = plan.execute_instances([_dev(torch, f) for f in fs])
    torch.cuda.synchronize()
    for k, (x, f, u) in enumerate(zip(xys, fs, us)):
        _check(u.cpu().numpy(), od.direct_sum(x, x, f), FP64_TOL, "instance %d" % k)
    plan.close()


def test_graph_replay_bit_exact(torch_mod, lf):
    torch = torch_mod
    xy = wl.clusters_on_background(np.random.default_rng(71), 10000, 1 << 16)
    f = _dev(torch, _loads(11, len(xy)))
    eager = _ctx(lf, max_leaf=32).plan(_dev(torch, xy))
    u0 = eager.execute(f).cpu().numpy()
    plan = _ctx(lf, max_leaf=32, graph=True).plan(_dev(torch, xy))
    for rep in range(3):
        u = plan.execute(f)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), u0), "replay %d" % rep
        torch.zeros(1000, device="cuda").sum().item()   # eager work between replays
    plan.close()
    eager.close()


@pytest.mark.parametrize("n,extent,max_leaf", [(1, 16, 8), (2, 1 << 20, 8), (8, 64, 8), (9, 64, 8),
                                               (40, 1 << 30, 4), (300, 1 << 12, 1)])
def test_degenerate_sizes(torch_mod, lf, n, extent, max_leaf):
    rng = np.random.default_rng(n)
    cells = set()
    while len(cells) < n:
        cells.add((int(rng.integers(0, extent)), int(rng.integers(0, extent))))
    xy = np.array(sorted(cells), dtype=np.int32)
    f = _loads(n, n) if n > 1 else np.array([1.0])
    u, plan = _solve(torch_mod, _ctx(lf, max_leaf=max_leaf), xy, f)
    ref = od.direct_sum(xy, xy, f)
    if n == 1:
        assert np.array_equal(u, ref)
    else:
        _check(u, ref, FP64_TOL, "n=%d" % n)
    plan.close()


def test_unsupported_entry_points(torch_mod, lf):
    torch = torch_mod
    ctx = _ctx(lf, max_leaf=32)
    xy = _dev(torch, np.array([[0, 0], [5, 3]], dtype=np.int32))
    f = _dev(torch, np.array([1.0, -1.0]))
    u = torch.empty(2, dtype=torch.float64, device="cuda")
    for call in (lambda: ctx.solve_static(xy, f, u), lambda: ctx.footprint_bytes(1000),
                 lambda: lf.Server(ctx)):
        with pytest.raises(lf.LfmmError) as e:
            call()
        assert e.value.status == -5   # LFMM_E_UNSUPPORTED


def test_clusters_full_size_sampled(torch_mod, lf):
    """2,000,000 clustered sources (64 Gaussian clusters, sigma 2,000, in 2^20 x 2^20) on the
    adaptive tree, FP64 and both mixed forms, compared on 2,000 sampled targets."""
    torch = torch_mod
    xy, f = wl.config_clusters()
    k = wl.sample_targets(3, len(xy), 2000)
    ref = od.direct_sum(xy[k], xy, f)
    for prec, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL), ("mixed-bf16", MIXED_TOL)):
        u, plan = _solve(torch, _ctx(lf, max_leaf=32, precision=prec), xy, f)
        info = plan.info()
        print(prec, {key: info[key] for key in ("n_boxes", "n_leaves", "near_pairs", "m2l_pairs", "m2p_terms",
                                                "p2l_terms")})
        _check(u[k], ref, tol, "clusters " + prec)
        plan.close()
