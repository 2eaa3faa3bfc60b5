"""ORACLE (test infrastructure only) -- the lattice fundamental solution phi.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
this package.  It shares no code with the GPU library.

What is computed (Gillman & Martinsson, "A fast solver for Poisson problems on infinite
regular lattices"):

* eq. (1.8): phi(m) = (2 pi)^-2 * integral over [-pi,pi]^2 of
  (cos(t1 m1 + t2 m2) - 1) / (4 sin^2(t1/2) + 4 sin^2(t2/2)) dt1 dt2,
  the fundamental solution of the 5-point operator of eq. (1.2): A phi = delta.
* Section 3.2: for small |m| the integral is evaluated by a two-step quadrature.  The square
  [-pi,pi]^2 is cut into n x n equal boxes with n odd and about |m| (one oscillation per
  box); every box except the centre one gets a 20 x 20 Gauss-Legendre rule; the centre box
  [-a,a]^2, a = pi/n, is written as the union of the annuli
  Omega_k = [-a 2^-k, a 2^-k]^2 minus [-a 2^-(k+1), a 2^-(k+1)]^2, k = 0, 1, 2, ...,
  each cut into eight rectangles with a 20 x 20 Gauss-Legendre rule on each.
* Section 3.1, eq. (3.1): for large |m| the expansion
  phi(m) ~ -(1/(2 pi)) (log|m| + gamma + log(8)/2)
           + (m1^4 - 6 m1^2 m2^2 + m2^4) / (24 pi |m|^6)
           + (43 m1^8 - 772 m1^6 m2^2 + 1570 m1^4 m2^4 - 772 m1^2 m2^6 + 43 m2^8) / (480 pi |m|^12).

Readings where the paper is silent or garbled (each is listed in the design notes):

* gamma is Euler's constant 0.5772156649015329; the six digits printed after eq. (3.1)
  contain a typo (they would shift phi by about 1.5e-6).
* n is the smallest odd integer >= max(3, |m|_inf) ("n about |m|", read per axis).
* The annulus index starts at k = 0 so that the annuli tile the whole centre box; the
  printed set definition dropped the minus signs of the inner corners.
* The paper accelerates the annulus series with Richardson extrapolation (about 14 terms).
  Here the series is summed directly for 40 terms: the integrand is bounded by |m|^2/2
  near the origin, so the neglected square [-a 2^-40, a 2^-40]^2 contributes < 1e-30.
* The paper's claim that the truncated expansion is accurate to 1e-12 for |m| > 30 does not
  hold (the error is about 0.15/|m|^6 on the axes, 2e-10 at |m| = 30).  The oracle uses the
  quadrature for |m|_inf <= 128 and the expansion only beyond, where the error is < 4e-14.
* The numerator cos(x) - 1 is evaluated as -2 sin^2(x/2), the same number without the
  cancellation near the origin.

Other lattice operators (the method carries over to other constant-coefficient difference
operators, Sections 1 and 3.1): eq. (1.8) with the symbol of the operator in the denominator,
by the same quadrature.  ``stencil=9`` is the isotropic 9-point operator
(20 u(m) - 4 (four neighbours) - (four diagonal neighbours)) / 6, whose symbol is
(20 - 8 cos t1 - 8 cos t2 - 4 cos t1 cos t2) / 6 = 4 (s1 + s2) - (8/3) s1 s2 with
s_i = sin^2(t_i / 2) (the 5-point symbol is 4 (s1 + s2)).  The oracle has no far-field
expansion for it: its values exist only inside the tabulated radius.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

# Euler's constant, the true value (the digits printed with eq. (3.1) are a typo).
EULER_GAMMA = 0.57721566490153286061

# Radius (infinity norm) up to which the oracle tabulates phi by quadrature.
TABLE_RADIUS = 128

_GL_X, _GL_W = np.polynomial.legendre.leggauss(20)
_N_ANNULI = 40


def _gauss(a: float, b: float):
    """20-point Gauss-Legendre nodes and weights on [a, b]."""
    h = 0.5 * (b - a)
    return a + h * (_GL_X + 1.0), h * _GL_W


def _symbol(t1, t2, stencil: int = 5):
    """Symbol of the lattice operator (the denominator of eq. 1.8), cancellation-free."""
    s1 = np.sin(0.5 * t1) ** 2
    s2 = np.sin(0.5 * t2) ** 2
    if stencil == 5:
        return 4.0 * s1 + 4.0 * s2
    if stencil == 9:
        return 4.0 * (s1 + s2) - (8.0 / 3.0) * s1 * s2
    raise ValueError("stencil must be 5 or 9")


def _integrand(t1, t2, m1: int, m2: int, stencil: int = 5):
    """The integrand of eq. (1.8), with cos(x) - 1 written as -2 sin^2(x/2)."""
    num = -2.0 * np.sin(0.5 * (m1 * t1 + m2 * t2)) ** 2
    return num / _symbol(t1, t2, stencil)


def box_count(m1: int, m2: int) -> int:
    """Number n of boxes per axis: odd, about |m|, at least 3 (Section 3.2)."""
    n = max(3, abs(int(m1)), abs(int(m2)))
    return n if n % 2 == 1 else n + 1


class _OuterGrid:
    """Tensor Gauss grid on the n x n boxes of [-pi,pi]^2, the centre box excluded."""

    def __init__(self, n: int, stencil: int = 5):
        self.stencil = stencil
        h = 2.0 * math.pi / n
        xs, ws = [], []
        for i in range(n):
            x, w = _gauss(-math.pi + i * h, -math.pi + (i + 1) * h)
            xs.append(x)
            ws.append(w)
        self.x = np.concatenate(xs)
        w = np.concatenate(ws)
        centre = np.zeros(n * 20, dtype=bool)
        c = (n - 1) // 2
        centre[c * 20:(c + 1) * 20] = True
        self.T1, self.T2 = np.meshgrid(self.x, self.x, indexing="ij")
        # quadrature weight times 1/denominator of the integrand, node by node
        den = _symbol(self.T1, self.T2, stencil)
        self.Wd = (w[:, None] * w[None, :]) / den
        # the centre box is integrated separately, by annuli
        self.Wd[np.ix_(centre, centre)] = 0.0
        self.buf = np.empty_like(self.T1)
        self.buf2 = np.empty_like(self.T1)
        self.a = math.pi / n

    def outer_sum(self, m1: int, m2: int) -> float:
        """Sum over the outer nodes of weight * integrand, integrand as in eq. (1.8)."""
        np.multiply(self.T1, 0.5 * m1, out=self.buf)
        np.multiply(self.T2, 0.5 * m2, out=self.buf2)
        np.add(self.buf, self.buf2, out=self.buf)
        np.sin(self.buf, out=self.buf)
        np.square(self.buf, out=self.buf)          # numerator = -2 sin^2((m.t)/2)
        np.multiply(self.buf, self.Wd, out=self.buf)
        # numpy's pairwise summation: deterministic, error ~ log2(#nodes) ulps
        return -2.0 * float(np.sum(self.buf))


def _annulus_rectangles(r: float):
    """The eight rectangles that tile [-r,r]^2 minus [-r/2,r/2]^2."""
    h = 0.5 * r
    return [
        (h, r, h, r), (-r, -h, h, r), (h, r, -r, -h), (-r, -h, -r, -h),   # corners
        (-h, h, h, r), (-h, h, -r, -h), (h, r, -h, h), (-r, -h, -h, h),   # edges
    ]


def _centre_box_integral(a: float, m1: int, m2: int, stencil: int = 5) -> float:
    """Integral of the eq. (1.8) integrand over [-a,a]^2 as a sum over annuli."""
    total = 0.0
    for k in range(_N_ANNULI):
        r = a * 2.0 ** (-k)
        part = 0.0
        for (x0, x1, y0, y1) in _annulus_rectangles(r):
            tx, wx = _gauss(x0, x1)
            ty, wy = _gauss(y0, y1)
            T1, T2 = np.meshgrid(tx, ty, indexing="ij")
            part += float(np.sum(wx[:, None] * wy[None, :] * _integrand(T1, T2, m1, m2, stencil)))
        total += part
    return total


def _phi_on_grid(grid: _OuterGrid, m1: int, m2: int) -> float:
    if m1 == 0 and m2 == 0:
        return 0.0
    outer = grid.outer_sum(m1, m2)
    centre = _centre_box_integral(grid.a, m1, m2, grid.stencil)
    return (outer + centre) / (4.0 * math.pi ** 2)


def phi_quadrature(m1: int, m2: int, stencil: int = 5) -> float:
    """phi(m) by the two-step quadrature of Section 3.2 (one value)."""
    return _phi_on_grid(_OuterGrid(box_count(m1, m2), stencil), int(m1), int(m2))


def _shell_worker(args):
    n, ms, stencil = args
    grid = _OuterGrid(n, stencil)
    return [(m1, m2, _phi_on_grid(grid, m1, m2)) for (m1, m2) in ms]


def octant_index(a: int, b: int) -> int:
    """Position of (a, b), 0 <= b <= a, in the octant table."""
    return a * (a + 1) // 2 + b


def octant_size(radius: int) -> int:
    return (radius + 1) * (radius + 2) // 2


def phi_table_quadrature(radius: int = TABLE_RADIUS, workers: int | None = None, stencil: int = 5) -> np.ndarray:
    """phi(a, b) for 0 <= b <= a <= radius by quadrature, in octant order.

    The octant suffices: phi is invariant under the eight symmetries of the square lattice,
    because the integrand of eq. (1.8) is.  Entries sharing a box count n share one grid.
    """
    groups: dict[int, list] = {}
    for a in range(radius + 1):
        for b in range(a + 1):
            groups.setdefault(box_count(a, b), []).append((a, b))
    jobs = []
    for n, ms in groups.items():
        step = max(1, len(ms) // 8)          # spread the big shells over workers
        for i in range(0, len(ms), step):
            jobs.append((n, ms[i:i + step], stencil))
    jobs.sort(key=lambda j: -j[0] * j[0] * len(j[1]))
    table = np.full(octant_size(radius), np.nan)
    workers = workers or min(8, os.cpu_count() or 1)
    if workers == 1:
        results = map(_shell_worker, jobs)
    else:
        ex = ProcessPoolExecutor(max_workers=workers)
        results = ex.map(_shell_worker, jobs)
    for chunk in results:
        for (a, b, v) in chunk:
            table[octant_index(a, b)] = v
    if workers != 1:
        ex.shutdown()
    return table


def phi_asymptotic(m1, m2):
    """Truncated expansion eq. (3.1), with the true Euler constant.  Vectorised; m != 0."""
    x = np.asarray(m1, dtype=np.float64)
    y = np.asarray(m2, dtype=np.float64)
    r2 = x * x + y * y
    c = x * x / r2
    s = y * y / r2
    lead = -(0.5 * np.log(r2) + EULER_GAMMA + 0.5 * math.log(8.0)) / (2.0 * math.pi)
    t4 = (c * c - 6.0 * c * s + s * s) / (24.0 * math.pi * r2)
    t8 = (43.0 * c ** 4 - 772.0 * c ** 3 * s + 1570.0 * c * c * s * s - 772.0 * c * s ** 3
          + 43.0 * s ** 4) / (480.0 * math.pi * r2 * r2)
    return lead + t4 + t8


_TABLE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "phi_quadrature_r128.txt")
_TABLE_FILE_9 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "phi9_quadrature_r128.txt")


def table_file(stencil: int = 5) -> str:
    return {5: _TABLE_FILE, 9: _TABLE_FILE_9}[stencil]


def load_table(path: str = _TABLE_FILE) -> np.ndarray:
    """The committed quadrature table (written by ``oracle/make_phi_table.py``)."""
    vals = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b, v = line.split()
            vals.append((int(a), int(b), float.fromhex(v)))
    radius = max(a for a, _, _ in vals)
    table = np.full(octant_size(radius), np.nan)
    for a, b, v in vals:
        table[octant_index(a, b)] = v
    if np.isnan(table).any():
        raise ValueError("incomplete phi table file")
    return table


def phi_lookup(m1, m2, table: np.ndarray, radius: int = TABLE_RADIUS):
    """phi at integer offsets: the quadrature table where |m|_inf <= radius, eq. (3.1) beyond."""
    m1 = np.abs(np.asarray(m1, dtype=np.int64))
    m2 = np.abs(np.asarray(m2, dtype=np.int64))
    a = np.maximum(m1, m2)
    b = np.minimum(m1, m2)
    out = np.empty(np.broadcast(a, b).shape, dtype=np.float64)
    near = a <= radius
    out[near] = table[(a[near] * (a[near] + 1)) // 2 + b[near]]
    far = ~near
    if np.any(far):
        out[far] = phi_asymptotic(a[far], b[far])
    return out
