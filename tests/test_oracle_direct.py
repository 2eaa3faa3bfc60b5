"""Pins for the oracle's direct sum u(t) = sum_s phi(t - s) f(s) (eq. 1.7)."""
import math

import numpy as np
import pytest

from oracle import direct as od
from oracle import phi as oph


def test_threads_reported():
    assert od.threads() >= 1


def test_brute_force_against_quadrature_values():
    # tiny input: every phi recomputed by the quadrature routine itself, summed in Python,
    # independent of the C code and of the stored table file
    rng = np.random.default_rng(7)
    src = rng.integers(-6, 7, size=(9, 2))
    f = rng.standard_normal(9)
    tgt = rng.integers(-8, 9, size=(5, 2))
    cache = {}

    def q(dx, dy):
        key = (max(abs(dx), abs(dy)), min(abs(dx), abs(dy)))
        if key not in cache:
            cache[key] = oph.phi_quadrature(*key)
        return cache[key]

    ref = np.array([sum(q(int(t[0] - s[0]), int(t[1] - s[1])) * fj for s, fj in zip(src, f))
                    for t in tgt])
    got = od.direct_sum(tgt, src, f)
    assert np.max(np.abs(got - ref)) <= 1e-14


def test_discrete_laplacian_of_potential_is_load():
    # A u = f (eq. 1.1) at every point of a window holding the sources, margin 2
    rng = np.random.default_rng(11)
    for trial in range(4):
        n = rng.integers(1, 21)
        cells = rng.choice(16 * 16, size=n, replace=False)
        src = np.stack([cells % 16, cells // 16], axis=1)
        f = rng.standard_normal(n)
        g = np.arange(-3, 19)
        X, Y = np.meshgrid(g, g, indexing="ij")
        tgt = np.stack([X.ravel(), Y.ravel()], axis=1)
        u = od.direct_sum(tgt, src, f).reshape(X.shape)
        Au = 4 * u[1:-1, 1:-1] - u[2:, 1:-1] - u[:-2, 1:-1] - u[1:-1, 2:] - u[1:-1, :-2]
        F = np.zeros_like(u)
        F[src[:, 0] + 3, src[:, 1] + 3] = f
        assert np.max(np.abs(Au - F[1:-1, 1:-1])) <= 1e-13 * max(1.0, np.max(np.abs(u)))


def test_laplacian_far_from_table():
    # same identity where every offset is beyond the table (expansion branch)
    rng = np.random.default_rng(5)
    src = rng.integers(0, 40, size=(12, 2))
    f = rng.standard_normal(12)
    g = np.arange(400, 406)
    X, Y = np.meshgrid(g, g, indexing="ij")
    u = od.direct_sum(np.stack([X.ravel(), Y.ravel()], 1), src, f).reshape(X.shape)
    Au = 4 * u[1:-1, 1:-1] - u[2:, 1:-1] - u[:-2, 1:-1] - u[1:-1, 2:] - u[1:-1, :-2]
    assert np.max(np.abs(Au)) <= 1e-13


@pytest.mark.parametrize("m", [(1, 0), (1, 1), (3, 2), (200, 200), (1000, 1000), (0, 777)])
def test_dipole_resistance(m):
    # loads +1 at a and -1 at a+m: u(a) - u(a+m) = -2 phi(m), the effective resistance of
    # the infinite unit-resistor grid; 1/2 for nearest neighbours, 2/pi across a diagonal
    a = np.array([17, -5])
    src = np.array([a, a + np.array(m)])
    u = od.direct_sum(src, src, np.array([1.0, -1.0]))
    R = u[0] - u[1]
    if m[0] == m[1]:
        n = m[0]
        exact = 2.0 * sum(1.0 / (2 * k - 1) for k in range(1, n + 1)) / math.pi
        assert abs(R - exact) <= 1e-13
    if m == (1, 0):
        assert abs(R - 0.5) <= 1e-15
    if m == (1, 1):
        assert abs(R - 2 / math.pi) <= 1e-15
    if m == (0, 777):
        assert abs(R + 2 * oph.phi_asymptotic(777, 0)) <= 1e-15


def test_far_field_matches_continuum_logarithm():
    # zero-sum loads: u(t) -> -(1/2pi) sum f log|t - s| + O(|t|^-2) far away (eq. 3.1)
    rng = np.random.default_rng(3)
    src = rng.integers(0, 32, size=(20, 2))
    f = rng.standard_normal(20)
    f -= f.mean()
    t = np.array([[5000, 3000], [-4000, 7000]])
    u = od.direct_sum(t, src, f)
    cont = np.array([-(f * np.log(np.hypot(*(tt - src).T))).sum() / (2 * math.pi) for tt in t])
    assert np.max(np.abs(u - cont)) <= 1e-7


def test_invariances():
    rng = np.random.default_rng(9)
    src = rng.integers(0, 300, size=(50, 2))
    f = rng.standard_normal(50)
    u = od.direct_sum(src, src, f)
    # integer translation
    shift = np.array([123456, -7890])
    assert np.array_equal(od.direct_sum(src + shift, src + shift, f), u)
    # a lattice symmetry (swap axes, flip one)
    rot = np.stack([src[:, 1], -src[:, 0]], axis=1)
    assert np.max(np.abs(od.direct_sum(rot, rot, f) - u)) <= 1e-13
    # linearity
    g = rng.standard_normal(50)
    lin = od.direct_sum(src, src, 2 * f - 3 * g)
    assert np.max(np.abs(lin - (2 * u - 3 * od.direct_sum(src, src, g)))) <= 1e-12
    # reciprocity <g, u_f> = <f, u_g>
    assert abs(g @ u - f @ od.direct_sum(src, src, g)) <= 1e-11
    # a zero-load source changes nothing
    src2 = np.vstack([src, [[-50, 40]]])
    f2 = np.append(f, 0.0)
    assert np.array_equal(od.direct_sum(src, src2, f2), u)


@pytest.mark.parametrize("m", [(129, 57), (-150, 149), (173, -88), (211, 5), (-256, -200), (300, 150),
                               (297, 296), (40, 290)])
def test_c_expansion_off_axis_against_reduced_integral(m):
    # the C direct sum's own phi beyond the table (eq. 3.1, off the axes and diagonal, signs
    # folded by the code under test) against the one-dimensional reduced integral of the remark
    # closing Section 3 at 30 digits; the truncation error of eq. 3.1 there is O(|m|^-6)
    import lattice_exact as le
    a, b = sorted((abs(m[0]), abs(m[1])), reverse=True)
    ref = le.phi_reduced_integral(a, b, digits=30)
    got = od.phi(np.array([m]))[0]
    assert abs(got - ref) <= 0.2 / math.hypot(*m) ** 6 + 2e-15
