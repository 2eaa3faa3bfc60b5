"""Pins for the oracle of Section 10 (lattice with inclusions; Dirichlet problem).

* A single modified bar a-b in a uniform field: by Thevenin's theorem the network seen from
  the bar's ends is a resistance R = -2 phi(a - b) in series with the unperturbed drop, so
  u(a) - u(b) = (v(a) - v(b)) / (1 + delta R).  With phi(e1) = -1/4 and phi(1, 1) = -1/pi
  this is a closed form.
* Many bars: the recovered u satisfies (A + B) u = 0 (eq. 10.1) on a window around them and
  tends to v far away (eq. 10.2).
* Dirichlet: u = D q with q from eq. 10.7 equals the solution of the discrete Dirichlet problem
  of eq. 10.5 computed by a sparse direct solve of A u = 0 with u = g on the boundary.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workloads as wl
from oracle import extensions as ox


@pytest.mark.parametrize("delta", [-1.0, -0.5, 0.7, 3.0])
def test_single_lattice_bar_closed_form(delta):
    bars = np.array([[0, 0, 1, 0]])
    nodes, mu = ox.inclusions_solve(bars, [delta], 1.0, 0.0)
    u = ox.inclusions_potential(bars, [delta], 1.0, 0.0, mu, [[0, 0], [1, 0]])
    assert abs((u[0] - u[1]) - (-1.0) / (1.0 + delta * 0.5)) <= 1e-14


@pytest.mark.parametrize("delta", [0.3, 2.0])
def test_single_added_diagonal_bar_closed_form(delta):
    bars = np.array([[5, -2, 6, -1]])
    c1, c2 = 1.0, 2.0
    nodes, mu = ox.inclusions_solve(bars, [delta], c1, c2)
    u = ox.inclusions_potential(bars, [delta], c1, c2, mu, [[5, -2], [6, -1]])
    dv = -(c1 + c2)
    assert abs((u[0] - u[1]) - dv / (1.0 + delta * 2.0 / math.pi)) <= 1e-13


def test_modified_lattice_equation_holds_on_window():
    rng = np.random.default_rng(3)
    bars, delta = wl.inclusion_bars(rng, 40, 12, origin=(-3, 4))
    c1, c2 = 0.7, -0.3
    nodes, mu = ox.inclusions_solve(bars, delta, c1, c2)
    g = np.arange(-8, 14)
    X, Y = np.meshgrid(g, g + 7, indexing="ij")
    win = np.stack([X.ravel(), Y.ravel()], axis=1)
    u = ox.inclusions_potential(bars, delta, c1, c2, mu, win).reshape(X.shape)
    Au = 4 * u[1:-1, 1:-1] - u[2:, 1:-1] - u[:-2, 1:-1] - u[1:-1, 2:] - u[1:-1, :-2]
    Bu = np.zeros_like(u)
    ix = lambda p: (p[0] - g[0], p[1] - g[0] - 7)
    for (a1, a2, b1, b2), d in zip(bars, delta):
        ia, ib = ix((a1, a2)), ix((b1, b2))
        Bu[ia] += d * (u[ia] - u[ib])
        Bu[ib] += d * (u[ib] - u[ia])
    res = Au + Bu[1:-1, 1:-1]
    assert np.max(np.abs(res)) <= 1e-11 * np.max(np.abs(u))
    # the printed recovery u = v - S(B v - mu) fails the same check
    load = ox.b_matrix(len(nodes), ox.inclusion_nodes(bars)[1], delta) @ (c1 * nodes[:, 0] + c2 * nodes[:, 1])
    from oracle import direct as od
    u_typo = (c1 * win[:, 0] + c2 * win[:, 1] - od.direct_sum(win, nodes, load - mu)).reshape(X.shape)
    Au_t = 4 * u_typo[1:-1, 1:-1] - u_typo[2:, 1:-1] - u_typo[:-2, 1:-1] - u_typo[1:-1, 2:] - u_typo[1:-1, :-2]
    assert np.max(np.abs(Au_t)) > 1e-3


def test_perturbation_decays_at_infinity():
    rng = np.random.default_rng(4)
    bars, delta = wl.inclusion_bars(rng, 30, 10)
    c1, c2 = 1.0, 0.5
    _, mu = ox.inclusions_solve(bars, delta, c1, c2)
    far = np.array([[1000, 0], [0, 1000], [100000, 0], [0, -100000]])
    u = ox.inclusions_potential(bars, delta, c1, c2, mu, far)
    w = u - (c1 * far[:, 0] + c2 * far[:, 1])
    # zero-sum loads: the perturbation decays like 1/|m|
    assert np.max(np.abs(w[2:])) <= 2e-2 * np.max(np.abs(w[:2]))


def _sparse_dirichlet(interior, gamma, g):
    idx = {tuple(p): k for k, p in enumerate(interior.tolist())}
    gd = {tuple(p): v for p, v in zip(gamma.tolist(), g)}
    rows, cols, vals = [], [], []
    b = np.zeros(len(interior))
    for k, (x, y) in enumerate(interior.tolist()):
        rows.append(k)
        cols.append(k)
        vals.append(4.0)
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            p = (x + dx, y + dy)
            if p in idx:
                rows.append(k)
                cols.append(idx[p])
                vals.append(-1.0)
            else:
                b[k] += gd[p]
    return spl.spsolve(sp.csr_matrix((vals, (rows, cols)), shape=(len(interior), len(interior))), b)


@pytest.mark.parametrize("shape", ["box", "wide_box", "lshape"])
def test_dirichlet_representation_solves_the_boundary_value_problem(shape):
    rng = np.random.default_rng(5)
    if shape == "box":
        gamma, codes, interior = wl.box_boundary(20, 20, origin=(3, -7))
    elif shape == "wide_box":
        gamma, codes, interior = wl.box_boundary(37, 9)
    else:
        gamma, codes, interior = wl.lshape_boundary(24, origin=(-50, 11))
    g = rng.standard_normal(len(gamma))
    q = ox.dirichlet_solve(gamma, codes, g)
    u_in = ox.d_apply(gamma, codes, q, interior)
    u_ref = _sparse_dirichlet(interior, gamma, g)
    assert np.max(np.abs(u_in - u_ref)) <= 1e-12 * np.max(np.abs(u_ref))
    assert np.max(np.abs(ox.d_apply(gamma, codes, q, gamma) - g)) <= 1e-12
    # the normal step of every boundary node leaves the domain
    inner = set(map(tuple, interior.tolist()))
    assert not any(tuple(p) in inner for p in (gamma + ox.NORMALS[codes]).tolist())
