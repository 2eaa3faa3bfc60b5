"""ORACLE (test infrastructure only) -- the two uses of the lattice convolution in Section 10.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
this module.  It shares no code with the GPU library.  Everything here is dense linear algebra
in FP64 on top of the oracle's phi (``oracle.direct.phi``) and direct sum of eq. (1.7).

Lattice with inclusions (Section 10.1, eq. 10.1-10.4).  A is the 5-point operator of eq. (1.2),
a sum over the lattice bars of (e_a - e_b)(e_a - e_b)^T.  The local modification B changes
bars: bar k joins nodes a_k, b_k and adds delta_k to its conductance (-1 removes a unit bar, a
bar between nodes that had none is added with delta_k > 0), so
    (B w)(a_k) += delta_k (w(a_k) - w(b_k)),   (B w)(b_k) += delta_k (w(b_k) - w(a_k)).
The problem (A + B) u = 0 with u -> v = c1 m1 + c2 m2 at infinity is solved as in the paper:
w = u - v, mu = B w, S = convolution with phi, and on the nodes touched by the bars
    mu + B S mu = -B S B v                                               (eq. 10.4)
after which
    u = v - S (B v + mu).
Reading: the paper prints the recovery as u = v - S(Bv - mu).  With its own definitions,
A w = -B v - B w = -(B v + mu) gives w = -S(B v + mu), so the sign in front of mu is read
as +; the (A + B) u = 0 pins of the tests fail with the printed sign.

Finite lattice, Dirichlet problem (Section 10.2, eq. 10.5-10.7).  For boundary nodes n in Gamma
with outward unit lattice normals nu(n) (n + nu(n) lies outside the domain), the
double-layer-like operator is read as
    [D q](m) = sum_{n in Gamma} [phi(m - n - nu(n)) - phi(m - n)] q(n),
the difference acting on the source variable n along its normal (eq. 10.6 is garbled in the
source: its sum over Gamma and the name of the density are lost).  A (D q) vanishes at every
node that is neither in Gamma nor an outside neighbour n + nu(n), so D q is discrete-harmonic
in the domain; the boundary condition u = g on Gamma is the equation of eq. 10.7,
    sum_{n in Gamma} d(m, n) q(n) = g(m),  m in Gamma.
The paper cites an O(N_Gamma) inversion that it does not describe; here it is solved densely.
"""
from __future__ import annotations

import numpy as np

from . import direct as od

NORMALS = np.array([[1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.int64)   # codes 0..3: +x, -x, +y, -y


def _phi_matrix(targets, sources) -> np.ndarray:
    """Dense matrix phi(t_i - s_j) (oracle phi, FP64)."""
    t = np.asarray(targets, dtype=np.int64)
    s = np.asarray(sources, dtype=np.int64)
    d = (t[:, None, :] - s[None, :, :]).reshape(-1, 2)
    return od.phi(d).reshape(len(t), len(s))


# ---- lattices with inclusions (Section 10.1) ------------------------------------------------

def inclusion_nodes(bars):
    """Distinct bar end points (Omega_inc) in first-appearance order, and each bar's two node
    indices.  bars: [n, 4] rows (a1, a2, b1, b2)."""
    bars = np.asarray(bars, dtype=np.int64).reshape(-1, 4)
    index, nodes = {}, []
    ends = np.empty((len(bars), 2), dtype=np.int64)
    for k, row in enumerate(bars):
        for e, p in enumerate(((int(row[0]), int(row[1])), (int(row[2]), int(row[3])))):
            if p not in index:
                index[p] = len(nodes)
                nodes.append(p)
            ends[k, e] = index[p]
    return np.array(nodes, dtype=np.int64).reshape(-1, 2), ends


def b_matrix(n_nodes: int, ends, delta) -> np.ndarray:
    """Dense B on the nodes: each bar adds delta (e_a - e_b)(e_a - e_b)^T."""
    B = np.zeros((n_nodes, n_nodes))
    for (a, b), d in zip(ends, np.asarray(delta, dtype=np.float64)):
        B[a, a] += d
        B[b, b] += d
        B[a, b] -= d
        B[b, a] -= d
    return B


def inclusions_solve(bars, delta, c1: float, c2: float):
    """mu on the nodes from eq. (10.4), solved densely.  Returns (nodes, mu)."""
    nodes, ends = inclusion_nodes(bars)
    B = b_matrix(len(nodes), ends, delta)
    S = _phi_matrix(nodes, nodes)
    v = c1 * nodes[:, 0] + c2 * nodes[:, 1]
    mu = np.linalg.solve(np.eye(len(nodes)) + B @ S, -(B @ (S @ (B @ v))))
    return nodes, mu


def inclusions_potential(bars, delta, c1: float, c2: float, mu, targets) -> np.ndarray:
    """u = v - S (B v + mu) at the targets (the recovery step after eq. 10.4)."""
    nodes, ends = inclusion_nodes(bars)
    B = b_matrix(len(nodes), ends, delta)
    v_nodes = c1 * nodes[:, 0] + c2 * nodes[:, 1]
    load = B @ v_nodes + np.asarray(mu, dtype=np.float64)
    t = np.asarray(targets, dtype=np.int64).reshape(-1, 2)
    return c1 * t[:, 0] + c2 * t[:, 1] - od.direct_sum(t, nodes, load)


# ---- Dirichlet problem on a finite lattice (Section 10.2) -----------------------------------

def dipole_sources(gamma, normal_codes):
    """Source points of D and the sign of each: +q at n + nu(n), -q at n."""
    g = np.asarray(gamma, dtype=np.int64).reshape(-1, 2)
    nu = NORMALS[np.asarray(normal_codes, dtype=np.int64)]
    return np.vstack([g + nu, g])


def d_apply(gamma, normal_codes, q, targets) -> np.ndarray:
    """[D q](t) by the direct sum of eq. (1.7) over the dipole sources."""
    q = np.asarray(q, dtype=np.float64)
    return od.direct_sum(np.asarray(targets, dtype=np.int64).reshape(-1, 2),
                         dipole_sources(gamma, normal_codes), np.concatenate([q, -q]))


def d_matrix(gamma, normal_codes) -> np.ndarray:
    """Dense d(m, n) of eq. 10.7 for m, n in Gamma."""
    g = np.asarray(gamma, dtype=np.int64).reshape(-1, 2)
    nu = NORMALS[np.asarray(normal_codes, dtype=np.int64)]
    return _phi_matrix(g, g + nu) - _phi_matrix(g, g)


def dirichlet_solve(gamma, normal_codes, g_values) -> np.ndarray:
    """q with D q = g on Gamma (eq. 10.7), solved densely."""
    return np.linalg.solve(d_matrix(gamma, normal_codes), np.asarray(g_values, dtype=np.float64))
