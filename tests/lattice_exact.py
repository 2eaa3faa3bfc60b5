"""Exact values of the lattice fundamental solution, for pinning the oracle.

Every phi(m) is r1 + r2/pi with r1, r2 rational.  Three facts fix all of them:

* phi(0) = 0 and A phi = delta (eq. 1.2 with eq. 1.8: the denominator of the integrand is
  the symbol of A, so A phi is the inverse Fourier transform of 1);
* invariance under the eight symmetries of the square lattice;
* the diagonal phi(n, n) = -(1/pi) sum_{k=1..n} 1/(2k-1), the classical diagonal of the
  square-lattice Green's function (its log growth matches eq. 3.1 along the diagonal).

Marching A phi = delta column by column in exact rationals then gives every value in the
octant 0 <= b <= a: for b < a at column a,
    phi(a+1, b) = 4 phi(a, b) - phi(a-1, b) - phi(a, b+1) - phi(a, |b-1|),
on the diagonal neighbour phi(a+1, a) = 2 phi(a, a) - phi(a, a-1), and phi(1, 0) = -1/4
from A phi = delta at the origin.  The march is exact in rationals but the two parts grow
like (3 + 2 sqrt 2)^a and cancel, so values are evaluated with many digits.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath


def diagonal(n: int):
    return (Fraction(0), -sum(Fraction(1, 2 * k - 1) for k in range(1, n + 1)))


def march(radius: int):
    """Dict (a, b) -> (r1, r2) with phi(a, b) = r1 + r2/pi, for 0 <= b <= a <= radius."""
    phi = {(0, 0): (Fraction(0), Fraction(0)),
           (1, 0): (Fraction(-1, 4), Fraction(0)),
           (1, 1): diagonal(1)}

    def get(a, b):
        a, b = abs(a), abs(b)
        if b > a:
            a, b = b, a
        return phi[(a, b)]

    def lin(*terms):
        r1 = sum((c * v[0] for c, v in terms), Fraction(0))
        r2 = sum((c * v[1] for c, v in terms), Fraction(0))
        return (r1, r2)

    for a in range(1, radius):
        for b in range(0, a):
            phi[(a + 1, b)] = lin((4, get(a, b)), (-1, get(a - 1, b)), (-1, get(a, b + 1)),
                                  (-1, get(a, b - 1)))
        phi[(a + 1, a)] = lin((2, get(a, a)), (-1, get(a, a - 1)))
        phi[(a + 1, a + 1)] = diagonal(a + 1)
    return phi


def evaluate(values, digits: int = 120):
    """Float values of the exact pairs, evaluated with ``digits`` significant digits."""
    out = {}
    with mpmath.workdps(digits):
        pi = mpmath.pi
        for k, (r1, r2) in values.items():
            v = mpmath.mpf(r1.numerator) / r1.denominator + (mpmath.mpf(r2.numerator) / r2.denominator) / pi
            out[k] = float(v)
    return out


def phi_reduced_integral(m1: int, m2: int, digits: int = 30) -> float:
    """phi(m) from the one-dimensional integral left after integrating eq. (1.8) in t1.

    With c = 4 - 2 cos t and lambda = (c - sqrt(c^2 - 4))/2 (the remark closing Section 3),
    phi(m) = (1/pi) int_0^pi (cos(m2 t) lambda^|m1| - 1) / sqrt(c^2 - 4) dt, |m1| >= |m2|.
    Evaluated with mpmath at ``digits`` digits, panels split at the oscillations of cos(m2 t).
    """
    a, b = abs(m1), abs(m2)
    if b > a:
        a, b = b, a
    if a == 0:
        return 0.0
    with mpmath.workdps(digits + 10):
        def g(t):
            if t == 0:
                return mpmath.mpf(-a) / 2      # the integrand's limit at t = 0
            # same quantities without cancellation: with s = sin(t/2), c - 2 = 4 s^2,
            # sqrt(c^2 - 4) = 4 s sqrt(1 + s^2) and lambda = (sqrt(1 + s^2) - s)^2
            s = mpmath.sin(t / 2)
            q = mpmath.sqrt(1 + s * s)
            rt = 4 * s * q
            lam = (q - s) ** 2
            return (mpmath.cos(b * t) * lam ** a - 1) / rt
        pts = [mpmath.mpf(0)]
        # geometric panels near 0 (lambda^a decays on the scale 1/a), uniform ones after
        h = mpmath.mpf(1) / (4 * a)
        while h < mpmath.pi / max(8, 2 * b):
            pts.append(h)
            h *= 2
        nun = max(8, 2 * b)
        start = pts[-1]
        for k in range(1, nun + 1):
            p = start + (mpmath.pi - start) * k / nun
            pts.append(p)
        val = mpmath.quad(g, pts) / mpmath.pi
        return float(val)


def phi9_reduced_integral(m1: int, m2: int, digits: int = 30) -> float:
    """phi of the isotropic 9-point operator (20 u - 4 (4 neighbours) - (4 diagonals)) / 6 from
    the one-dimensional integral left after integrating eq. (1.8) in t1: its symbol is
    (alpha - beta cos t1) / 6 with alpha = 20 - 8 cos t2, beta = 8 + 4 cos t2, and the t1
    integral of cos(k t1) / (alpha - beta cos t1) is 2 pi lambda^k / sqrt(alpha^2 - beta^2),
    lambda = (alpha - sqrt(alpha^2 - beta^2)) / beta, so that
    phi(m) = (6/pi) int_0^pi (cos(m2 t) lambda^|m1| - 1) / sqrt(alpha^2 - beta^2) dt, |m1| >= |m2|.
    Evaluated with mpmath at ``digits`` digits (extra working digits absorb the cancellation
    near t = 0)."""
    a, b = abs(m1), abs(m2)
    if b > a:
        a, b = b, a
    if a == 0:
        return 0.0
    with mpmath.workdps(2 * digits + 20):
        def g(t):
            if t == 0:
                return mpmath.mpf(-a) / 12     # the integrand's limit at t = 0 (beta(0) = 12)
            # with s = sin(t/2): alpha = 12 + 16 s^2, beta = 12 - 8 s^2, alpha - beta = 24 s^2 and
            # alpha + beta = 24 + 8 s^2, so sqrt(alpha^2 - beta^2) = s sqrt(24 (24 + 8 s^2))
            s = mpmath.sin(t / 2)
            al = 12 + 16 * s * s
            be = 12 - 8 * s * s
            rt = s * mpmath.sqrt(24 * (24 + 8 * s * s))
            lam = (al - rt) / be
            return (mpmath.cos(b * t) * lam ** a - 1) / rt
        pts = [mpmath.mpf(0)]
        h = mpmath.mpf(1) / (4 * a)
        while h < mpmath.pi / max(8, 2 * b):
            pts.append(h)
            h *= 2
        nun = max(8, 2 * b)
        start = pts[-1]
        for k in range(1, nun + 1):
            pts.append(start + (mpmath.pi - start) * k / nun)
        val = 6 * mpmath.quad(g, pts) / mpmath.pi
        return float(val)
