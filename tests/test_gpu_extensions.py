"""GPU parity of the Section 10 applications against the dense FP64 oracle (oracle.extensions):
the lattice with inclusions (eq. 10.4 by GMRES with S applied by a resident plan, then the
recovered potential) and the Dirichlet problem (D applied by the FMM, eq. 10.7 by GMRES, the
potential at interior nodes).

Bar: relative l2 and max-norm errors <= 1e-10 against the oracle (the FP64 target), with GMRES
run to a relative residual of 1e-13, well below it (the dense systems have condition numbers
near 10, so residual and error agree to that factor).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import extensions as ox

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def _errs(u, ref):
    return (float(np.linalg.norm(u - ref) / np.linalg.norm(ref)),
            float(np.max(np.abs(u - ref)) / np.max(np.abs(ref))))


@pytest.mark.parametrize("delta", [-1.0, 0.7])
def test_single_bar_closed_form(torch_mod, ctx, delta):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    inc = lf.Inclusions(ctx, [[0, 0, 1, 0]], [delta])
    mu, st = inc.solve(1.0, 0.0, tol=1e-14)
    u = inc.potential(1.0, 0.0, mu, _dev(torch, np.array([[0, 0], [1, 0]], np.int32))).cpu().numpy()
    assert abs((u[0] - u[1]) + 1.0 / (1.0 + 0.5 * delta)) <= 1e-12
    inc.close()


@pytest.mark.parametrize("n_bars,side", [(400, 60), (2500, 220)])
def test_inclusions_against_oracle(torch_mod, ctx, n_bars, side):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(700 + n_bars)
    bars, delta = wl.inclusion_bars(rng, n_bars, side, origin=(-side // 2, 1000))
    c1, c2 = 0.8, -0.45
    inc = lf.Inclusions(ctx, bars, delta)
    nodes_ref, mu_ref = ox.inclusions_solve(bars, delta, c1, c2)
    assert np.array_equal(inc.nodes, nodes_ref)     # same node order (first appearance)
    mu, st = inc.solve(c1, c2, tol=1e-13)
    print("inclusions %d bars, %d nodes: %d iterations, residual %.2e" % (n_bars, len(inc.nodes), st["iterations"],
                                                                        st["rel_residual"]))
    assert st["converged"] == 1
    l2, mx = _errs(mu.cpu().numpy(), mu_ref)
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    # the potential on a window over the inclusions and far away
    g = np.arange(-side // 2 - 5, side // 2 + 5, 3)
    X, Y = np.meshgrid(g, g + 1000 + side // 2, indexing="ij")
    tgt = np.vstack([np.stack([X.ravel(), Y.ravel()], axis=1), [[10 ** 6, -3], [-40000, 2 * 10 ** 5]]]).astype(np.int32)
    u = inc.potential(c1, c2, mu, _dev(torch, tgt)).cpu().numpy()
    ref = ox.inclusions_potential(bars, delta, c1, c2, mu_ref, tgt)
    v = c1 * tgt[:, 0] + c2 * tgt[:, 1]
    w, wref = (u - v)[:-2], (ref - v)[:-2]
    l2, mx = _errs(w, wref)         # the perturbation u - v on the window, the part the solver computes
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    # far away u is v to the last digits (|v| ~ 1e5 .. 1e6): compare u itself there
    assert np.all(np.abs(u[-2:] - ref[-2:]) <= 4e-16 * np.abs(v[-2:]) + TOL * np.max(np.abs(wref)))
    inc.close()


@pytest.mark.parametrize("shape", ["box", "lshape"])
def test_dirichlet_against_oracle(torch_mod, ctx, shape):
    import paper_1105_3505_amd as lf
    torch = torch_mod
    rng = np.random.default_rng(710)
    if shape == "box":
        gamma, codes, interior = wl.box_boundary(300, 170, origin=(-1000, 77))
    else:
        gamma, codes, interior = wl.lshape_boundary(180, origin=(5, 5))
    dirp = lf.Dirichlet(ctx, gamma, codes)
    # D applied by the FMM against the direct sum
    q0 = rng.standard_normal(len(gamma))
    d0 = dirp.apply(_dev(torch, q0)).cpu().numpy()
    l2, mx = _errs(d0, ox.d_apply(gamma, codes, q0, gamma))
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    # eq. 10.7 by GMRES against the dense solve
    g = np.sin(0.01 * gamma[:, 0]) + np.cos(0.013 * gamma[:, 1]) + 0.1 * rng.standard_normal(len(gamma))
    q, st = dirp.solve(_dev(torch, g), tol=1e-13)
    q_ref = ox.dirichlet_solve(gamma, codes, g)
    print("dirichlet %s: %d boundary nodes, %d iterations, residual %.2e"
          % (shape, len(gamma), st["iterations"], st["rel_residual"]))
    assert st["converged"] == 1
    l2, mx = _errs(q.cpu().numpy(), q_ref)
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    # the potential inside, at sampled interior nodes
    idx = wl.sample_targets(711, len(interior), 3000)
    u = dirp.potential(q, _dev(torch, interior[idx])).cpu().numpy()
    l2, mx = _errs(u, ox.d_apply(gamma, codes, q_ref, interior[idx]))
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    dirp.close()
