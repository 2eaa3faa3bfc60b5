"""Pins for the oracle's phi (quadrature table of Section 3.2 + expansion eq. 3.1).

Each check compares against something the oracle does not compute itself: closed forms,
the exact rational march of A phi = delta, the diagonal formula, the one-dimensional
reduced integral evaluated at 30 digits, and the analytic size of the expansion's error.
"""
import math

import numpy as np
import pytest

import lattice_exact as le
from oracle import phi as oph


@pytest.fixture(scope="module")
def table():
    return oph.load_table()


@pytest.fixture(scope="module")
def exact64():
    return le.evaluate(le.march(64), digits=160)


def tab(table, a, b):
    return oph.phi_lookup(a, b, table).item()


CLOSED = {
    (0, 0): 0.0,
    (1, 0): -0.25,
    (1, 1): -1 / math.pi,
    (2, 0): -1 + 2 / math.pi,
    (2, 1): 0.25 - 2 / math.pi,
    (2, 2): -4 / (3 * math.pi),
    (3, 0): -17 / 4 + 12 / math.pi,
    (3, 1): 2 - 23 / (3 * math.pi),
    (3, 2): -0.25 - 2 / (3 * math.pi),
    (3, 3): -23 / (15 * math.pi),
}


def test_table_complete_and_finite(table):
    assert table.shape == (oph.octant_size(oph.TABLE_RADIUS),)
    assert np.all(np.isfinite(table))


@pytest.mark.parametrize("m,val", sorted(CLOSED.items()))
def test_closed_forms(table, m, val):
    # phi(0)=0, phi(e1)=-1/4, phi(1,1)=-1/pi and the rest follow from A phi = delta
    assert abs(tab(table, *m) - val) <= 1e-15


def test_quadrature_reproduces_closed_forms_directly():
    # the quadrature routine itself (not the stored file)
    for m, val in CLOSED.items():
        assert abs(oph.phi_quadrature(*m) - val) <= 1e-15


def test_symmetries_of_lookup(table):
    rng = np.random.default_rng(0)
    m = rng.integers(-300, 301, size=(200, 2))
    base = oph.phi_lookup(m[:, 0], m[:, 1], table)
    for sx, sy, swap in [(-1, 1, 0), (1, -1, 0), (-1, -1, 0), (1, 1, 1), (-1, 1, 1)]:
        a, b = sx * m[:, 0], sy * m[:, 1]
        if swap:
            a, b = b, a
        assert np.array_equal(oph.phi_lookup(a, b, table), base)


def test_exact_march_radius_64(table, exact64):
    # the octant out to |m|_inf = 64 against the exact rational values of A phi = delta
    err = max(abs(tab(table, a, b) - v) for (a, b), v in exact64.items())
    assert err <= ENTRY_TOL, err


# Tolerances: a table entry sums up to 6.7e6 quadrature terms pairwise, so its rounding is
# about log2(6.7e6) ulps of the summed magnitude, ~2e-15 at |m| ~ 128 (values near 1.5).
ENTRY_TOL = 3e-15


def test_diagonal_formula_to_table_edge(table):
    for n in range(1, oph.TABLE_RADIUS + 1):
        exact = -sum(1.0 / (2 * k - 1) for k in range(1, n + 1)) / math.pi
        assert abs(tab(table, n, n) - exact) <= ENTRY_TOL, n


def test_a_phi_equals_delta_on_whole_table(table):
    # (A phi)(m) = 4 phi(m) - sum of the 4 neighbours = delta(m), at every table point whose
    # neighbours are in the table as well
    R = oph.TABLE_RADIUS - 1
    a, b = np.meshgrid(np.arange(R + 1), np.arange(R + 1), indexing="ij")
    keep = b <= a
    a, b = a[keep], b[keep]
    res = (4 * oph.phi_lookup(a, b, table) - oph.phi_lookup(a + 1, b, table)
           - oph.phi_lookup(a - 1, b, table) - oph.phi_lookup(a, b + 1, table)
           - oph.phi_lookup(a, b - 1, table))
    delta = ((a == 0) & (b == 0)).astype(float)
    # the residual weighs five entries by 4 + 1 + 1 + 1 + 1
    assert np.max(np.abs(res - delta)) <= 8 * ENTRY_TOL


def test_a_phi_equals_delta_across_switch(table):
    # beyond the table the expansion (error O(|m|^-6)) takes over; its discrete Laplacian
    # residual is far below the accuracy target
    pts = [(128, 0), (128, 64), (128, 128), (129, 3), (150, 40), (200, 200), (1000, 7)]
    for (x, y) in pts:
        r = (4 * tab(table, x, y) - tab(table, x + 1, y) - tab(table, x - 1, y)
             - tab(table, x, y + 1) - tab(table, x, y - 1))
        assert abs(r) <= 1e-13, (x, y, r)


@pytest.mark.parametrize("m", [(31, 0), (37, 11), (45, 45), (64, 3), (90, 77), (127, 1), (128, 128)])
def test_reduced_integral_spot_points(table, m):
    # the one-dimensional reduced integral (remark at the end of Section 3), 30 digits
    ref = le.phi_reduced_integral(*m, digits=30)
    assert abs(tab(table, *m) - ref) <= ENTRY_TOL


@pytest.mark.parametrize("m", [(129, 0), (160, 33), (200, 200), (333, 1)])
def test_expansion_beyond_table_against_reduced_integral(table, m):
    # beyond radius 128 the oracle uses eq. (3.1); its error there is O(|m|^-6)
    ref = le.phi_reduced_integral(*m, digits=30)
    r = math.hypot(*m)
    assert abs(tab(table, *m) - ref) <= 0.2 / r ** 6 + 1e-15


def test_expansion_error_decays_like_r6(table):
    # inside the table, table minus expansion shrinks like |m|^-6 along the axis (the first
    # dropped term), pinning the expansion's coefficients and Euler's constant
    errs = []
    for n in (32, 64, 128):
        errs.append(abs(tab(table, n, 0) - oph.phi_asymptotic(n, 0)))
    assert errs[0] > 1e-11 and errs[2] < 5e-14
    ratio1, ratio2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 50 < ratio1 < 80 and 50 < ratio2 < 80      # 2^6 = 64


def test_printed_gamma_would_fail():
    # the six digits printed with eq. (3.1) are off by ~9.5e-6; the oracle's constant is
    # the true one, which the exact diagonal confirms
    n = 100
    exact = -sum(1.0 / (2 * k - 1) for k in range(1, n + 1)) / math.pi
    assert abs(oph.phi_asymptotic(n, n) - exact) < 1e-13
    lead_typo = -(math.log(n * math.sqrt(2)) + 0.577206 + 0.5 * math.log(8)) / (2 * math.pi)
    assert abs(lead_typo - exact) > 1e-6


def test_stored_table_matches_quadrature_script(table):
    # a sample of entries recomputed by the quadrature routine must equal the stored file
    for (a, b) in [(0, 0), (1, 0), (5, 2), (17, 16), (40, 9), (101, 50)]:
        assert oph.phi_quadrature(a, b) == tab(table, a, b)
