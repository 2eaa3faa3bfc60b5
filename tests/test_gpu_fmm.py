"""GPU parity: the HIP lattice FMM and direct kernel against the FP64 oracle (eq. 1.7).

Tolerance: relative l2 error <= 1e-10 over the compared targets for the FMM (the FP64
accuracy target), <= 1e-13 for the direct kernel (same sum, only phi tables and rounding
order differ).
"""
import math

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


def _fmm(torch, ctx, xy, f):
    plan = ctx.plan(_dev(torch, xy))
    u = plan.execute(_dev(torch, f))
    torch.cuda.synchronize()
    return u.cpu().numpy(), plan


def _rel(u, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(u - ref) / (den if den > 0 else 1.0))


def _maxrel(u, ref):
    """max |u - u_ref| / max |u_ref|: the max-norm error reported beside the l2 one."""
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(u - ref)) / (den if den > 0 else 1.0))


def test_direct_kernel_matches_oracle(torch_mod, ctx):
    torch = torch_mod
    rng = np.random.default_rng(21)
    src = rng.integers(0, 400, size=(700, 2)).astype(np.int32)
    tgt = rng.integers(-100, 500, size=(300, 2)).astype(np.int32)
    f = rng.standard_normal(700)
    u = ctx.direct(_dev(torch, tgt), _dev(torch, src), _dev(torch, f))
    torch.cuda.synchronize()
    ref = od.direct_sum(tgt, src, f)
    assert _rel(u.cpu().numpy(), ref) <= 1e-13


def test_small_uniform_all_targets(torch_mod, ctx):
    xy, f = wl.config_small_uniform()
    u, plan = _fmm(torch_mod, ctx, xy, f)
    ref = od.direct_sum(xy, xy, f)
    err = _rel(u, ref)
    info = plan.info()
    print("n=1000 leaf level %d side %d rel err %.3e" % (info["leaf_level"], info["leaf_side"], err))
    assert info["leaf_level"] >= 2          # the far-field passes ran
    assert err <= FMM_TOL and _maxrel(u, ref) <= FMM_TOL


@pytest.mark.parametrize("n,side,seed", [(1, 16, 1), (2, 16, 2), (17, 64, 3), (64, 64, 4), (65, 64, 5),
                                         (300, 100, 6), (2000, 181, 7), (5000, 2000, 8), (20000, 600, 9)])
def test_uniform_sizes_all_targets(torch_mod, ctx, n, side, seed):
    rng = np.random.default_rng(seed)
    xy = wl.uniform_box(rng, n, side, origin=(-side // 3, 1000 * seed))
    f = wl.zero_sum_loads(rng.standard_normal(n)) if n > 1 else np.array([1.5])
    u, _ = _fmm(torch_mod, ctx, xy, f)
    ref = od.direct_sum(xy, xy, f)
    if n == 1:
        assert u[0] == 0.0                  # phi(0) = 0: no self term
    else:
        assert _rel(u, ref) <= FMM_TOL and _maxrel(u, ref) <= FMM_TOL


def test_clustered_points(torch_mod, ctx):
    rng = np.random.default_rng(12)
    centres = rng.uniform(200, 3800, size=(6, 2))
    xy = wl.gaussian_clusters(rng, 8000, centres, 60.0, 4096)
    f = wl.zero_sum_loads(rng.uniform(-1, 1, 8000))
    u, _ = _fmm(torch_mod, ctx, xy, f)
    ref = od.direct_sum(xy, xy, f)
    assert _rel(u, ref) <= FMM_TOL


def test_nonzero_total_load(torch_mod, ctx):
    # the library returns the finite sum for any loads
    rng = np.random.default_rng(13)
    xy = wl.uniform_box(rng, 3000, 300)
    f = rng.uniform(0.5, 1.5, 3000)
    u, _ = _fmm(torch_mod, ctx, xy, f)
    ref = od.direct_sum(xy, xy, f)
    assert _rel(u, ref) <= FMM_TOL


def test_duplicate_points_superpose(torch_mod, ctx):
    rng = np.random.default_rng(14)
    base = wl.uniform_box(rng, 500, 120)
    xy = np.vstack([base, base[:200]])
    f = rng.standard_normal(700)
    u, _ = _fmm(torch_mod, ctx, xy, f)
    ref = od.direct_sum(xy, xy, f)
    assert _rel(u, ref) <= FMM_TOL


def test_deterministic_and_plan_reuse(torch_mod, ctx):
    torch = torch_mod
    rng = np.random.default_rng(15)
    xy = wl.uniform_box(rng, 10000, 500)
    f = wl.zero_sum_loads(rng.standard_normal(10000))
    g = wl.zero_sum_loads(rng.standard_normal(10000))
    plan = ctx.plan(_dev(torch, xy))
    u1 = plan.execute(_dev(torch, f)).cpu().numpy()
    u2 = plan.execute(_dev(torch, f)).cpu().numpy()
    ug = plan.execute(_dev(torch, g)).cpu().numpy()
    assert np.array_equal(u1, u2)
    ul = plan.execute(_dev(torch, 2 * f - 3 * g)).cpu().numpy()
    assert _rel(ul, 2 * u1 - 3 * ug) <= 1e-12
    # reciprocity <g, u_f> = <f, u_g> (T_tfi = T_ofs^T, Section 7)
    assert abs(g @ u1 - f @ ug) <= 1e-10 * np.linalg.norm(g) * np.linalg.norm(u1)


def test_translation_and_symmetry(torch_mod, ctx):
    rng = np.random.default_rng(16)
    xy = wl.uniform_box(rng, 6000, 400)
    f = wl.zero_sum_loads(rng.standard_normal(6000))
    u, _ = _fmm(torch_mod, ctx, xy, f)
    # an integer translation moves the root box with the points: same arithmetic
    ut, _ = _fmm(torch_mod, ctx, xy + np.array([123457, -98765], dtype=np.int32), f)
    assert np.array_equal(u, ut)
    rot = np.stack([xy[:, 1], -xy[:, 0]], axis=1).astype(np.int32)
    ur, _ = _fmm(torch_mod, ctx, rot, f)
    assert _rel(ur, u) <= 2 * FMM_TOL


def test_dipole_effective_resistance(torch_mod, ctx):
    # +1 at a, -1 at a+m amid zero-load points: u(a) - u(a+m) = -2 phi(m); across a diagonal
    # of n cells that is (2/pi) sum_{k<=n} 1/(2k-1)
    rng = np.random.default_rng(17)
    n = 300
    xy = wl.uniform_box(rng, 5000, 1500)
    a = xy[0]
    xy[1] = a + n
    f = np.zeros(5000)
    f[0], f[1] = 1.0, -1.0
    u, _ = _fmm(torch_mod, ctx, xy, f)
    exact = 2.0 * sum(1.0 / (2 * k - 1) for k in range(1, n + 1)) / math.pi
    assert abs((u[0] - u[1]) - exact) <= 1e-10


def test_extent_out_of_range(torch_mod, ctx):
    import paper_1105_3505_amd as lf
    xy = np.array([[-(2 ** 31) + 5, 0], [2 ** 31 - 5, 0]], dtype=np.int32)
    with pytest.raises(lf.LfmmError) as e:
        ctx.plan(_dev(torch_mod, xy))
    assert e.value.status == -2


@pytest.mark.slow
def test_large_uniform_sampled(torch_mod, ctx):
    # 1,000,000 sources uniform in a 4096 x 4096 box; 2,000 sampled targets
    xy, f = wl.config_large_uniform()
    u, plan = _fmm(torch_mod, ctx, xy, f)
    idx = wl.sample_targets(20, len(xy), 2000)
    ref = od.direct_sum(xy[idx], xy, f)
    err = _rel(u[idx], ref)
    info = plan.info()
    mx = _maxrel(u[idx], ref)
    print("n=1e6 leaf level %d side %d near pairs %d m2l pairs %d rel err %.3e max %.3e"
          % (info["leaf_level"], info["leaf_side"], info["near_pairs"], info["m2l_pairs"], err, mx))
    assert err <= FMM_TOL and mx <= FMM_TOL


@pytest.mark.slow
def test_clusters_sampled(torch_mod, ctx):
    # 2,000,000 sources in 64 Gaussian clusters over a 2^20 x 2^20 region (leaf side 128: the
    # near field reads the device octant table); 500 sampled targets
    xy, f = wl.config_clusters()
    u, plan = _fmm(torch_mod, ctx, xy, f)
    info = plan.info()
    assert info["leaf_side"] >= 64
    idx = wl.sample_targets(21, len(xy), 500)
    ref = od.direct_sum(xy[idx], xy, f)
    err = _rel(u[idx], ref)
    mx = _maxrel(u[idx], ref)
    print("n=2e6 clusters leaf level %d side %d near pairs %d m2l pairs %d rel err %.3e max %.3e"
          % (info["leaf_level"], info["leaf_side"], info["near_pairs"], info["m2l_pairs"], err, mx))
    assert err <= FMM_TOL and mx <= FMM_TOL


@pytest.mark.parametrize("max_leaf", [8, 16, 32, 128, 256])
def test_leaf_sizes(torch_mod, max_leaf):
    # leaf sides from 2 to 64: window table, quadrant table and global-table near fields
    import paper_1105_3505_amd as lf
    ctx = lf.Context(0, max_leaf=max_leaf)
    rng = np.random.default_rng(50 + max_leaf)
    xy = wl.uniform_box(rng, 12000, 440)
    f = wl.zero_sum_loads(rng.standard_normal(12000))
    u, plan = _fmm(torch_mod, ctx, xy, f)
    assert _rel(u, od.direct_sum(xy, xy, f)) <= FMM_TOL
    plan.close()
    ctx.close()


@pytest.mark.parametrize("precision", ["mixed", "mixed-bf16"])
def test_mixed_precision_m2l(torch_mod, precision):
    # FP32 hi/lo (or three-part bf16) matrix-core M2L; everything else FP64; target 1e-7
    import paper_1105_3505_amd as lf
    ctx = lf.Context(0, precision=precision)
    for seed, n, side in [(61, 1000, 256), (62, 30000, 700)]:
        rng = np.random.default_rng(seed)
        xy = wl.uniform_box(rng, n, side)
        f = wl.zero_sum_loads(rng.standard_normal(n))
        u, _ = _fmm(torch_mod, ctx, xy, f)
        ref = od.direct_sum(xy, xy, f)
        err, mx = _rel(u, ref), _maxrel(u, ref)
        print("%s n=%d rel err %.3e max %.3e" % (precision, n, err, mx))
        assert err <= 1e-7 and mx <= 1e-7
    ctx.close()
