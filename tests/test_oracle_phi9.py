"""Pins for the oracle's phi of the isotropic 9-point operator
A9 u(m) = (20 u(m) - 4 (sum of the 4 neighbours) - (sum of the 4 diagonal neighbours)) / 6,
computed by the two-step quadrature of Section 3.2 with the operator's symbol in eq. (1.8):

* A9 phi = delta over the whole table (the denominator of eq. 1.8 is the symbol of A9);
* spot values against the one-dimensional reduced integral (the t1 integral done in closed
  form, evaluated with mpmath at 30 digits): an independent route;
* the direct sum solves A9 u = f on a window around its sources;
* far out, phi + log|m| / (2 pi) settles to a constant faster than |m|^-2 (the symbol is
  |t|^2 - |t|^4 / 12 + O(|t|^6): its |t|^4 term is isotropic, so no |m|^-2 correction).
"""
import math

import numpy as np
import pytest

import lattice_exact as le
from oracle import direct as od
from oracle import phi as oph

R = oph.TABLE_RADIUS


@pytest.fixture(scope="module")
def table():
    return od.table(9)


def tab(t, a, b):
    a, b = abs(a), abs(b)
    if b > a:
        a, b = b, a
    return t[a * (a + 1) // 2 + b]


def test_table_complete(table):
    assert len(table) == (R + 1) * (R + 2) // 2 and np.all(np.isfinite(table))
    assert table[0] == 0.0


def test_a9_phi_equals_delta(table):
    worst = 0.0
    for a in range(0, R):
        for b in range(0, a + 1):
            nb = tab(table, a + 1, b) + tab(table, a - 1, b) + tab(table, a, b + 1) + tab(table, a, b - 1)
            dg = (tab(table, a + 1, b + 1) + tab(table, a - 1, b + 1) + tab(table, a + 1, b - 1)
                  + tab(table, a - 1, b - 1))
            r = (20 * tab(table, a, b) - 4 * nb - dg) / 6 - (1.0 if (a, b) == (0, 0) else 0.0)
            worst = max(worst, abs(r))
    assert worst <= 2e-14


@pytest.mark.parametrize("m", [(1, 0), (1, 1), (2, 1), (9, 4), (33, 0), (50, 50), (101, 77), (128, 3)])
def test_reduced_integral_spot_points(table, m):
    assert abs(tab(table, *m) - le.phi9_reduced_integral(*m, digits=30)) <= 4e-15


def test_direct_sum_solves_the_9_point_equation():
    rng = np.random.default_rng(19)
    cells = rng.choice(14 * 14, size=12, replace=False)
    src = np.stack([cells % 14, cells // 14], axis=1)
    f = rng.standard_normal(12)
    g = np.arange(-3, 17)
    X, Y = np.meshgrid(g, g, indexing="ij")
    u = od.direct_sum(np.stack([X.ravel(), Y.ravel()], axis=1), src, f, stencil=9).reshape(X.shape)
    A9u = (20 * u[1:-1, 1:-1] - 4 * (u[2:, 1:-1] + u[:-2, 1:-1] + u[1:-1, 2:] + u[1:-1, :-2])
           - (u[2:, 2:] + u[:-2, 2:] + u[2:, :-2] + u[:-2, :-2])) / 6
    F = np.zeros_like(u)
    F[src[:, 0] + 3, src[:, 1] + 3] = f
    assert np.max(np.abs(A9u - F[1:-1, 1:-1])) <= 1e-13 * max(1.0, np.max(np.abs(u)))


def test_log_growth_without_r2_correction(table):
    # g(m) = phi + log|m| / (2 pi) along the axis and the diagonal: differences between radii
    # shrink like |m|^-4 (a |m|^-2 correction would make them shrink 4x slower)
    def g(a, b):
        return tab(table, a, b) + math.log(math.hypot(a, b)) / (2 * math.pi)
    for d in ((1, 0), (1, 1)):
        e1 = abs(g(32 * d[0], 32 * d[1]) - g(64 * d[0], 64 * d[1]))
        e2 = abs(g(64 * d[0], 64 * d[1]) - g(128 * d[0], 128 * d[1]))
        assert e2 < e1 / 10


def test_beyond_table_is_refused():
    with pytest.raises(ValueError):
        od.direct_sum([[0, 0]], [[200, 0]], [1.0], stencil=9)
    assert np.isnan(od.phi([[300, 1]], stencil=9)[0])
