"""Seeded point/load generators for the lattice Poisson workloads.

The paper's experiments (Section 9) use synthetic geometries: loads drawn uniformly at
random in an n-by-n box of Z^2, dense boxes and points on a circle.  The generators below
produce those shapes plus the clustered and multi-instance mixes used for measurement.

Every generator returns ``(xy, f)`` with ``xy`` an int32 array of shape [N, 2] (column 0
is the first lattice coordinate m1, column 1 is m2) and ``f`` a float64 array of N loads
whose exact sum is zero (the well-posedness condition of Section 1).

Zero sum is made exact, not approximate: loads are mean-subtracted, rounded to integer
multiples of 2^-32, and the last one is set to minus the sum of the others.  All values are
then exactly representable, so sum(f) == 0 holds in exact arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

_QUANT = 2.0 ** 32


def zero_sum_loads(raw: np.ndarray) -> np.ndarray:
    """Mean-subtract ``raw`` and quantise so that the loads sum to exactly zero."""
    raw = np.asarray(raw, dtype=np.float64)
    if raw.size == 0:
        return raw.copy()
    centred = raw - raw.mean()
    k = np.rint(centred * _QUANT).astype(np.int64)
    k[-1] = -int(k[:-1].sum())
    return k.astype(np.float64) / _QUANT


def uniform_box(rng: np.random.Generator, n: int, side: int, origin=(0, 0)) -> np.ndarray:
    """``n`` distinct lattice cells drawn uniformly (without replacement) from a side x side box."""
    side = int(side)
    total = side * side
    if n > total:
        raise ValueError("more points than cells")
    if total <= 4 * n:
        cells = rng.choice(total, size=n, replace=False)
    else:
        # sparse box: draws with replacement, later duplicates rejected (the same law as
        # drawing without replacement, at a cost in n rather than in side^2)
        cells = np.empty(0, dtype=np.int64)
        while len(cells) < n:
            need = n - len(cells)
            cand = np.concatenate([cells, rng.integers(0, total, size=need + need // 8 + 16)])
            _, first = np.unique(cand, return_index=True)
            first.sort()
            cells = cand[first][:n]
    xy = np.empty((n, 2), dtype=np.int64)
    xy[:, 0] = cells % side + origin[0]
    xy[:, 1] = cells // side + origin[1]
    return xy.astype(np.int32)


def gaussian_clusters(rng: np.random.Generator, n: int, centres: np.ndarray, sigma: float,
                      extent: int) -> np.ndarray:
    """``n`` distinct lattice points, split evenly over Gaussian clusters.

    Each point is round(centre + sigma * g) with g standard normal in 2-D, clipped to
    [0, extent).  Duplicate cells are redrawn until ``n`` distinct points exist.
    """
    centres = np.asarray(centres, dtype=np.float64)
    k = len(centres)
    per = np.full(k, n // k, dtype=np.int64)
    per[: n - per.sum()] += 1
    extent = int(extent)
    keys = np.empty(0, dtype=np.int64)       # accepted cells, in acceptance order
    need = per.copy()
    while need.sum() > 0:
        draws = []
        for c in range(k):
            if need[c] == 0:
                continue
            g = rng.standard_normal((int(need[c]), 2))
            p = np.rint(centres[c] + sigma * g).astype(np.int64)
            np.clip(p, 0, extent - 1, out=p)
            draws.append((c, p[:, 0] * extent + p[:, 1]))
        cand = np.concatenate([keys] + [d for _, d in draws])
        owner = np.concatenate([np.full(len(keys), -1)] + [np.full(len(d), c) for c, d in draws])
        _, first = np.unique(cand, return_index=True)
        keep = np.zeros(len(cand), dtype=bool)
        keep[first] = True
        keep[: len(keys)] = True                 # earlier acceptances always stay
        new_mask = keep[len(keys):]
        new_owner = owner[len(keys):]
        keys = cand[keep]
        for c in range(k):
            need[c] -= int(np.count_nonzero(new_mask & (new_owner == c)))
    xy = np.empty((n, 2), dtype=np.int64)
    xy[:, 0] = keys // extent
    xy[:, 1] = keys % extent
    return xy.astype(np.int32)


# ----------------------------------------------------------------------------------------
# Named workloads.  Sizes follow the measurement configurations of the build: a small
# uniform case the oracle sums in seconds, a 1e6-source uniform case, a clustered case in
# a 2^20 region, a batch of 512 uneven instances and a stream of serving requests.
# ----------------------------------------------------------------------------------------

def clusters_on_background(rng: np.random.Generator, n: int, extent: int, n_clusters: int = 3,
                           sigma: float = 0.0, background: float = 0.3) -> np.ndarray:
    """``n`` distinct lattice points in [0, extent)^2: a fraction ``background`` uniform over the
    whole square, the rest in Gaussian clusters (sigma default extent / 400) centred in its
    middle 60 %.  Densities differ by orders of magnitude, so an adaptive tree puts its leaves
    on many levels."""
    extent = int(extent)
    sigma = float(sigma) if sigma > 0 else extent / 400.0
    nb = int(round(background * n))
    centres = rng.uniform(0.2 * extent, 0.8 * extent, size=(n_clusters, 2))
    core = gaussian_clusters(rng, n - nb, centres, sigma, extent)
    taken = set((core[:, 0].astype(np.int64) * extent + core[:, 1]).tolist())
    bg = []
    while len(bg) < nb:
        c = rng.integers(0, extent, size=(2 * (nb - len(bg)) + 8, 2))
        for x, y in c.tolist():
            k = x * extent + y
            if k not in taken:
                taken.add(k)
                bg.append((x, y))
                if len(bg) == nb:
                    break
    xy = np.concatenate([core, np.array(bg, dtype=np.int32).reshape(-1, 2)]).astype(np.int32)
    return xy[rng.permutation(len(xy))]


def config_small_uniform(seed: int = 1, n: int = 1000, side: int = 256):
    """1,000 distinct sources uniform in a 256 x 256 box, N(0,1) loads, zero sum."""
    rng = np.random.default_rng(seed)
    xy = uniform_box(rng, n, side)
    f = zero_sum_loads(rng.standard_normal(n))
    return xy, f


def config_large_uniform(seed: int = 2, n: int = 1_000_000, side: int = 4096):
    """1,000,000 distinct sources uniform in a 4096 x 4096 box, N(0,1) loads, zero sum."""
    rng = np.random.default_rng(seed)
    xy = uniform_box(rng, n, side)
    f = zero_sum_loads(rng.standard_normal(n))
    return xy, f


def config_clusters(seed: int = 3, n: int = 2_000_000, n_clusters: int = 64,
                    sigma: float = 2000.0, extent: int = 1 << 20, margin: float = 6000.0):
    """Sources in Gaussian clusters (sigma = 2,000) inside a 2^20 x 2^20 region, U(-1,1) loads."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(margin, extent - margin, size=(n_clusters, 2))
    xy = gaussian_clusters(rng, n, centres, sigma, extent)
    f = zero_sum_loads(rng.uniform(-1.0, 1.0, size=n))
    return xy, f


def batched_sizes(seed: int = 4, n_inst: int = 512, lo: float = 1e3, hi: float = 1e5):
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_inst))).astype(np.int64)


def config_batched_instance(seed: int, i: int, n_inst: int = 512, lo: float = 1e3, hi: float = 1e5):
    """Instance i of config_batched: uniform in a box of side ceil(4 sqrt N), zero-sum loads."""
    n = int(batched_sizes(seed, n_inst, lo, hi)[i])
    rng = np.random.default_rng([seed, i])
    side = int(math.ceil(4.0 * math.sqrt(n)))
    xy = uniform_box(rng, n, side)
    f = zero_sum_loads(rng.standard_normal(n))
    return xy, f


def config_batched(seed: int = 4, n_inst: int = 512, lo: float = 1e3, hi: float = 1e5):
    """Independent uniform instances with log-uniform sizes, each in a box of side ceil(4 sqrt N)."""
    return [config_batched_instance(seed, i, n_inst, lo, hi) for i in range(n_inst)]


def serving_request_size(seed: int, index: int, lo: float = 1e2, hi: float = 1e6) -> int:
    """Size of request ``index`` of ``config_serving_request`` (same draws), without its points."""
    rng = np.random.default_rng([seed, index])
    return max(int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi))))), 2)


def config_serving_request(seed: int, index: int, lo: float = 1e2, hi: float = 1e6):
    """One serving request: log-uniform size, uniform or 8-cluster layout chosen by the seed."""
    rng = np.random.default_rng([seed, index])
    n = int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    n = max(n, 2)
    if rng.uniform() < 0.5:
        side = int(math.ceil(4.0 * math.sqrt(n)))
        xy = uniform_box(rng, n, side)
        layout = "uniform"
    else:
        sigma = math.sqrt(n)
        box = int(math.ceil(16.0 * math.sqrt(n)))
        centres = rng.uniform(3 * sigma, box - 3 * sigma, size=(8, 2))
        xy = gaussian_clusters(rng, n, centres, sigma, box)
        layout = "clusters"
    f = zero_sum_loads(rng.standard_normal(n))
    return xy, f, layout


def sample_targets(seed: int, n: int, k: int) -> np.ndarray:
    """Indices of ``min(k, n)`` targets sampled without replacement, sorted."""
    rng = np.random.default_rng(seed)
    k = min(int(k), int(n))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# ----------------------------------------------------------------------------------------
# Geometries of the two applications of the lattice convolution (lattice with inclusions,
# Dirichlet problem on a finite lattice).  Points and coefficients only.
# ----------------------------------------------------------------------------------------

def inclusion_bars(rng: np.random.Generator, n_bars: int, side: int, origin=(0, 0),
                   frac_removed: float = 0.15, frac_added: float = 0.15):
    """``n_bars`` distinct bar modifications in a side x side box.

    Returns ``(bars, delta)``: bars [n, 4] int32 rows (a1, a2, b1, b2), the two nodes of the
    bar; delta [n] float64, the change of its conductance.  Lattice bars (unit horizontal or
    vertical) are removed (delta = -1), weakened (delta in (-0.9, 0)) or strengthened (delta
    in (0, 3)); added bars join diagonal neighbours (delta in (0.1, 2)).  No node loses more
    than one of its bars, so no part of the lattice is cut off and (A + B) stays invertible
    on decaying functions.
    """
    seen, removed = set(), {}
    bars, delta = [], []
    ox, oy = int(origin[0]), int(origin[1])
    while len(bars) < n_bars:
        x, y = int(rng.integers(0, side)), int(rng.integers(0, side))
        r = rng.uniform()
        if r < frac_added:
            dx, dy = (1, 1) if rng.uniform() < 0.5 else (1, -1)
            d = float(rng.uniform(0.1, 2.0))
            kind = "add"
        else:
            dx, dy = (1, 0) if rng.uniform() < 0.5 else (0, 1)
            kind = "remove" if r < frac_added + frac_removed else "change"
            d = -1.0 if kind == "remove" else float(rng.choice([rng.uniform(-0.9, -0.05), rng.uniform(0.05, 3.0)]))
        a, b = (ox + x, oy + y), (ox + x + dx, oy + y + dy)
        key = (a, b)
        if key in seen:
            continue
        if kind == "remove" and (removed.get(a, 0) >= 1 or removed.get(b, 0) >= 1):
            continue
        seen.add(key)
        if kind == "remove":
            removed[a] = removed.get(a, 0) + 1
            removed[b] = removed.get(b, 0) + 1
        bars.append((a[0], a[1], b[0], b[1]))
        delta.append(d)
    return np.array(bars, dtype=np.int32), np.array(delta, dtype=np.float64)


# normal codes of the Dirichlet boundary: 0: +x, 1: -x, 2: +y, 3: -y (outward)
def box_boundary(n1: int, n2: int, origin=(0, 0)):
    """Boundary of the box [0, n1] x [0, n2] without its corners: the nodes next to the
    interior (0, n1) x (0, n2), with outward normal codes.  Returns (gamma [m, 2] int32,
    codes [m] int8, interior [k, 2] int32)."""
    ox, oy = int(origin[0]), int(origin[1])
    g, c = [], []
    for t in range(1, n2):
        g += [(ox, oy + t), (ox + n1, oy + t)]
        c += [1, 0]
    for t in range(1, n1):
        g += [(ox + t, oy), (ox + t, oy + n2)]
        c += [3, 2]
    xs, ys = np.meshgrid(np.arange(1, n1) + ox, np.arange(1, n2) + oy, indexing="ij")
    interior = np.stack([xs.ravel(), ys.ravel()], axis=1)
    return np.array(g, dtype=np.int32), np.array(c, dtype=np.int8), interior.astype(np.int32)


def lshape_boundary(n: int, origin=(0, 0)):
    """L-shaped domain: the interior of [0, n]^2 minus the quadrant [n/2, n]^2; its boundary
    nodes (outside the domain, next to it) with outward normal codes chosen so that the
    normal step leaves the domain.  Returns (gamma, codes, interior)."""
    h = n // 2
    inside = lambda x, y: 0 < x < n and 0 < y < n and not (x >= h and y >= h)
    interior = [(x, y) for x in range(n + 1) for y in range(n + 1) if inside(x, y)]
    iset = set(interior)
    steps = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    g, c = [], []
    for x in range(-1, n + 2):
        for y in range(-1, n + 2):
            if (x, y) in iset:
                continue
            nb = [k for k, (dx, dy) in enumerate(steps) if (x + dx, y + dy) in iset]
            if not nb:
                continue
            out = [k for k, (dx, dy) in enumerate(steps) if (x + dx, y + dy) not in iset and k ^ 1 in nb]
            code = out[0] if out else nb[0] ^ 1
            g.append((x, y))
            c.append(code)
    ox, oy = int(origin[0]), int(origin[1])
    gam = np.array(g, dtype=np.int64) + [ox, oy]
    inter = np.array(interior, dtype=np.int64) + [ox, oy]
    return gam.astype(np.int32), np.array(c, dtype=np.int8), inter.astype(np.int32)
