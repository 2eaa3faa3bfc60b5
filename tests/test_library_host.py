"""Host-side checks of the C-ABI library (no GPU): symbols, phi and the operators.

The library's phi comes from the reduced one-dimensional integral (remark closing Section
3); the oracle's from the two-step quadrature of Section 3.2.  The operators are checked
against their defining properties (Sections 5 and 7) with the oracle's phi.
"""
import ctypes

import numpy as np
import pytest

import paper_1105_3505_amd as lf
from oracle import direct as od
from oracle import phi as oph


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(lf.library_path())
    names = lf.exported_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_no_device_reports_status():
    # without a GPU in this process, creating a context must fail with a status, not crash
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(lf.LfmmError) as e:
        lf.Context(0)
    assert e.value.status == -6


def test_host_phi_matches_oracle_table():
    a, b = np.meshgrid(np.arange(129), np.arange(129), indexing="ij")
    keep = b <= a
    m = np.stack([a[keep], b[keep]], axis=1)
    lib = lf.host_phi(m)
    ref = oph.phi_lookup(m[:, 0], m[:, 1], oph.load_table())
    assert np.max(np.abs(lib - ref)) <= 5e-15


def test_host_phi_symmetry_and_far_field():
    rng = np.random.default_rng(1)
    m = rng.integers(-5000, 5001, size=(500, 2))
    v = lf.host_phi(m)
    assert np.array_equal(v, lf.host_phi(-m))
    assert np.array_equal(v, lf.host_phi(m[:, ::-1]))
    ref = od.phi(m)
    # the oracle stops eq. (3.1) after the |m|^-4 terms, whose remainder against the Section 3.2
    # quadrature is below 3.5e-14 (128 / |m|)^6; the library adds fitted |m|^-6 terms
    r = np.hypot(m[:, 0], m[:, 1]).astype(np.float64)
    bound = 5e-15 + 3.5e-14 * np.minimum(1.0, 128.0 / r) ** 6
    assert np.all(np.abs(v - ref) <= bound)


def test_host_phi_closed_forms():
    v = lf.host_phi([[0, 0], [1, 0], [1, 1], [0, -1]])
    assert v[0] == 0.0
    assert abs(v[1] + 0.25) <= 2e-16 and abs(v[3] + 0.25) <= 2e-16
    assert abs(v[2] + 1 / np.pi) <= 2e-16


@pytest.mark.parametrize("side", [1, 2, 4, 16, 32])
def test_operators_shapes_and_skeletons(side):
    ops = lf.HostOperators(side, 4)
    prev_rank = None
    for h in range(4):
        s, r = ops.level(h)
        assert s == side << h
        assert 1 <= r <= 48
        sk = ops.skeleton(h)
        assert sk.shape == (r, 2) and sk.min() >= 0 and sk.max() < s
        if h == 0:
            # leaf skeleton lies on the box boundary (candidates of Section 5)
            on_edge = (sk == 0) | (sk == s - 1)
            assert np.all(on_edge.any(axis=1))
        else:
            assert ops.ofo(h, 0).shape == (r, prev_rank)
        prev_rank = r
    T = ops.leaf()
    assert T.shape == (ops.level(0)[1], side * side)


def _far_targets(s, rng, k):
    # points outside the concentric box of side 3s (well separated, Section 4.2)
    out = []
    while len(out) < k:
        p = rng.integers(-12 * s, 13 * s, size=2)
        if not (-s <= p[0] <= 2 * s - 1 and -s <= p[1] <= 2 * s - 1):
            out.append(p)
    return np.array(out)


def test_leaf_outgoing_expansion_reproduces_far_field():
    # eq. (5.1): sources anywhere in the leaf, equivalent charges at the skeleton
    s = 16
    ops = lf.HostOperators(s, 1)
    rng = np.random.default_rng(2)
    cells = rng.choice(s * s, size=40, replace=False)
    src = np.stack([cells % s, cells // s], axis=1)
    q = rng.standard_normal(40)
    qhat = ops.leaf()[:, cells] @ q
    tgt = _far_targets(s, rng, 300)
    ref = od.direct_sum(tgt, src, q)
    app = od.direct_sum(tgt, ops.skeleton(0), qhat)
    assert np.max(np.abs(app - ref)) <= 1e-11 * np.max(np.abs(ref))
    # the charge sum is kept exactly enough for the log far field
    assert abs(qhat.sum() - q.sum()) <= 1e-12


def test_outgoing_from_outgoing_reproduces_far_field():
    # Section 7: parent expansion from the four children's expansions
    s = 8
    ops = lf.HostOperators(s, 3)
    rng = np.random.default_rng(3)
    for h in (1, 2):
        side, _ = ops.level(h)
        half, _ = ops.level(h - 1)
        sk_c = ops.skeleton(h - 1)
        src, q, qhat = [], [], np.zeros(ops.level(h)[1])
        for c in range(4):
            off = np.array([(c & 1) * half, (c >> 1) * half])
            qc = rng.standard_normal(len(sk_c))
            src.append(sk_c + off)
            q.append(qc)
            qhat += ops.ofo(h, c) @ qc
        src, q = np.vstack(src), np.concatenate(q)
        tgt = _far_targets(side, rng, 300)
        ref = od.direct_sum(tgt, src, q)
        app = od.direct_sum(tgt, ops.skeleton(h), qhat)
        assert np.max(np.abs(app - ref)) <= 1e-11 * np.max(np.abs(ref)), h


def test_bad_arguments_return_status():
    with pytest.raises(lf.LfmmError):
        lf.HostOperators(3, 2)          # not a power of two
    with pytest.raises(lf.LfmmError):
        lf.HostOperators(16, 0)
    with pytest.raises(lf.LfmmError):
        lf.HostOperators(16, 2, eps=-1.0)


def test_host_phi9_matches_oracle_table():
    # the library's 9-point phi (one-dimensional reduced integral) against the oracle's (two-step
    # quadrature of Section 3.2 with the 9-point symbol): independent routes
    a, b = np.meshgrid(np.arange(129), np.arange(129), indexing="ij")
    keep = b <= a
    m = np.stack([a[keep], b[keep]], axis=1)
    lib = lf.host_phi(m, stencil=9)
    ref = od.phi(m, stencil=9)
    assert np.max(np.abs(lib - ref)) <= 5e-15


@pytest.mark.parametrize("m", [(129, 0), (140, 139), (181, 60), (256, 1), (400, 399), (1000, 10)])
def test_host_phi9_far_field_against_reduced_integral(m):
    # beyond the table the library uses its fitted expansion; the reference is the reduced
    # integral at 30 digits (tests/lattice_exact.py)
    import lattice_exact as le
    assert abs(lf.host_phi([m], stencil=9)[0] - le.phi9_reduced_integral(*m, digits=30)) <= 2e-15


def test_host_phi9_operator_equation_across_the_switch():
    def A9(x, y):
        pts = [[x, y], [x + 1, y], [x - 1, y], [x, y + 1], [x, y - 1],
               [x + 1, y + 1], [x - 1, y + 1], [x + 1, y - 1], [x - 1, y - 1]]
        v = lf.host_phi(pts, stencil=9)
        return (20 * v[0] - 4 * v[1:5].sum() - v[5:].sum()) / 6
    assert abs(A9(0, 0) - 1.0) <= 1e-14
    for p in [(128, 0), (128, 77), (129, 129), (150, 2), (700, 300)]:
        assert abs(A9(*p)) <= 1e-14, p


def test_leaf_outgoing_expansion_9_point():
    # eq. (5.1) for the 9-point operator: the skeleton charges reproduce the leaf's far field
    s = 8
    ops = lf.HostOperators(s, 1, stencil=9)
    rng = np.random.default_rng(4)
    cells = rng.choice(s * s, size=30, replace=False)
    src = np.stack([cells % s, cells // s], axis=1)
    q = rng.standard_normal(30)
    qhat = ops.leaf()[:, cells] @ q
    # well-separated targets inside the oracle's 9-point table radius
    tgt = rng.integers(-56, 72, size=(2000, 2))
    far = np.max(np.abs(tgt - s // 2), axis=1) >= 2 * s
    tgt = tgt[far][:300]
    ref = od.direct_sum(tgt, src, q, stencil=9)
    app = od.direct_sum(tgt, ops.skeleton(0), qhat, stencil=9)
    assert np.max(np.abs(app - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_skeleton_ranks_follow_table1():
    """Table 1 (tests/golden/table1_ranks.txt): skeleton sizes for eps = 1e-6 .. 1e-13 of the
    continuum kernel are 19-21, 27-29, 36-37, 49-51 whatever the box size.  The lattice
    operators of boxes of side 32 to 256 need the same numbers within a few points (their ID
    also keeps the total charge, one more column, and its tolerance is relative to the first
    pivot), and the rank does not grow with the box."""
    import golden_fixtures as gf
    table = gf.table1_ranks()
    for eps, ref in table.items():
        ops = lf.HostOperators(32, 4, eps=eps, max_rank=64)
        ranks = [ops.level(h)[1] for h in range(4)]
        ops.close()
        assert min(ref) - 2 <= min(ranks) and max(ranks) <= max(ref) + 4, (eps, ranks, ref)
        assert max(ranks) - min(ranks) <= 3


def _opset_arrays(ops, n_levels):
    out = [np.array([ops.level(h) for h in range(n_levels)])]
    out += [ops.skeleton(h) for h in range(n_levels)]
    out += [ops.ofo(h, c) for h in range(1, n_levels) for c in range(4)]
    out.append(ops.leaf())
    return out


def test_operator_cache_round_trip(tmp_path, monkeypatch):
    """LFMM_CACHE_DIR: the first build writes the operator set, later builds read it back bit for
    bit; a damaged file is rebuilt (and rewritten), never trusted."""
    monkeypatch.delenv("LFMM_CACHE_DIR", raising=False)
    ref = lf.HostOperators(32, 3)
    want = _opset_arrays(ref, 3)
    ref.close()
    monkeypatch.setenv("LFMM_CACHE_DIR", str(tmp_path))
    stamps = []
    for _ in range(2):   # build and store, then load (the file is not rewritten)
        ops = lf.HostOperators(32, 3)
        got = _opset_arrays(ops, 3)
        ops.close()
        assert all(np.array_equal(a, b) for a, b in zip(want, got))
        files = sorted(tmp_path.glob("opset_*.bin"))
        assert len(files) == 1
        stamps.append(files[0].stat().st_mtime_ns)
    assert stamps[0] == stamps[1]
    size = files[0].stat().st_size
    files[0].write_bytes(files[0].read_bytes()[:-100])
    ops = lf.HostOperators(32, 3)
    got = _opset_arrays(ops, 3)
    ops.close()
    assert all(np.array_equal(a, b) for a, b in zip(want, got))
    assert files[0].stat().st_size == size
    other = lf.HostOperators(32, 3, eps=1e-10)   # another key: another file
    other.close()
    assert len(list(tmp_path.glob("opset_*.bin"))) == 2
