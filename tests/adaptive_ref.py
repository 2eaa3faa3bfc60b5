"""Brute-force reference of the adaptive quadtree and its lists (test infrastructure).

Written from the definitions, box pair by box pair, with no traversal: Section 6 (closing
paragraph) refines a box while it holds more than N_leaf points; the far field then goes
through the lists of Carrier, Greengard and Rokhlin (1988):

* U(tau), tau a leaf: the leaves whose closed squares meet tau's (tau itself included);
* V(tau): boxes of tau's level that do not touch tau and whose parents touch tau's parent;
* W(tau), tau a leaf: boxes finer than tau that do not touch it but whose parents do;
* X(tau): leaves coarser than tau that touch tau's parent but not tau.

With ``direct_max`` (the library uses its skeleton size, 48), a box holding at most that many
points takes no expansion route: a W box that small joins U (its points summed directly,
fewer terms than its skeleton), and a box that small keeps no X list, the leaves below it
taking its X entries into their U lists.

Boxes are given as arrays over the non-empty boxes of a uniform-depth quadtree (level,
integer coordinates at that level, parent index, point count), the layout the library
exports.  ``coverage`` checks the property the lists exist for: every (target leaf, source
leaf) pair is accounted for exactly once, by U directly or through one ancestor pair of the
other three lists.
"""
from __future__ import annotations

import numpy as np

PRUNED, INNER, LEAF = 0, 1, 2


def compact_bits(v):
    v = np.asarray(v, dtype=np.uint64)
    out = np.zeros(v.shape, dtype=np.int64)
    for b in range(32):
        out |= ((v >> np.uint64(2 * b)) & np.uint64(1)).astype(np.int64) << b
    return out


def roles(level, parent, count, max_leaf, leaf_level):
    """Role of every box: in the adaptive tree when its parent holds more than max_leaf points
    (roots always), and a leaf of it when it holds at most max_leaf points or lies on the
    finest level.  max_leaf and leaf_level are per box (its instance's)."""
    level = np.asarray(level)
    parent = np.asarray(parent)
    count = np.asarray(count)
    pc = np.where(parent >= 0, count[np.maximum(parent, 0)], np.iinfo(np.int64).max)
    member = (level == 0) | (parent < 0) | (pc > max_leaf)
    leaf = (count <= max_leaf) | (level >= leaf_level)
    return np.where(member, np.where(leaf, LEAF, INNER), PRUNED).astype(np.int8)


def _touch(la, xa, ya, lb, xb, yb):
    """Closed squares of boxes a and b (vectorised over b) meet."""
    fine = np.maximum(la, lb)
    sa = 1 << (fine - la)
    sb = 1 << (fine - lb)
    ax0, ax1 = xa * sa, (xa + 1) * sa
    ay0, ay1 = ya * sa, (ya + 1) * sa
    bx0, bx1 = xb * sb, (xb + 1) * sb
    by0, by1 = yb * sb, (yb + 1) * sb
    return (ax0 <= bx1) & (bx0 <= ax1) & (ay0 <= by1) & (by0 <= ay1)


def _overlap(la, xa, ya, lb, xb, yb):
    fine = np.maximum(la, lb)
    sa = 1 << (fine - la)
    sb = 1 << (fine - lb)
    return ((xa * sa < (xb + 1) * sb) & (xb * sb < (xa + 1) * sa) &
            (ya * sa < (yb + 1) * sb) & (yb * sb < (ya + 1) * sa))


def lists(level, x, y, parent, inst, role, count=None, direct_max=None):
    """U, V, W, X of every box as sorted lists of box indices (empty where undefined); with
    direct_max, small W boxes and the X lists of small boxes move to U (see above)."""
    level = np.asarray(level, dtype=np.int64)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    parent = np.asarray(parent)
    inst = np.asarray(inst)
    role = np.asarray(role)
    nb = len(level)
    U, V, W, X = ([[] for _ in range(nb)] for _ in range(4))
    member = role != PRUNED
    for t in range(nb):
        if role[t] == PRUNED:
            continue
        same = (inst == inst[t]) & member
        lt, xt, yt = level[t], x[t], y[t]
        touch_t = _touch(lt, xt, yt, level, x, y) & ~_overlap(lt, xt, yt, level, x, y)
        if role[t] == LEAF:
            U[t] = sorted([t] + list(np.nonzero(same & (role == LEAF) & touch_t)[0]))
            par = np.maximum(parent, 0)
            ptouch = (parent >= 0) & _touch(lt, xt, yt, level[par], x[par], y[par]) & \
                ~_overlap(lt, xt, yt, level[par], x[par], y[par])
            W[t] = sorted(np.nonzero(same & (level > lt) & ~touch_t & ~_overlap(lt, xt, yt, level, x, y) &
                                     ptouch)[0].tolist())
        if lt >= 2:
            p = parent[t]
            lp, xp, yp = level[p], x[p], y[p]
            par = np.maximum(parent, 0)
            pp_touch = (parent >= 0) & (_touch(lp, xp, yp, level[par], x[par], y[par]))
            V[t] = sorted(np.nonzero(same & (level == lt) & ~touch_t & (np.arange(nb) != t) & pp_touch)[0].tolist())
            touch_p = _touch(lp, xp, yp, level, x, y) & ~_overlap(lp, xp, yp, level, x, y)
            X[t] = sorted(np.nonzero(same & (role == LEAF) & (level < lt) & touch_p & ~touch_t)[0].tolist())
    if direct_max is None:
        return U, V, W, X
    count = np.asarray(count)
    small = count <= direct_max
    X2 = [x if not small[t] else [] for t, x in enumerate(X)]
    U2, W2 = [], []
    for t in range(nb):
        if role[t] != LEAF:
            U2.append([])
            W2.append([])
            continue
        extra = [d for d in W[t] if small[d]]
        a = t
        while a >= 0 and level[a] >= 2 and small[a]:
            extra += X[a]
            a = parent[a]
        U2.append(sorted(U[t] + extra))
        W2.append([d for d in W[t] if not small[d]])
    return U2, V, W2, X2


def coverage(parent, role, U, V, W, X, inst):
    """Times each (target leaf, source leaf) pair of one instance is accounted for: U
    directly; V, W and X through the pair (ancestor-or-self of the target, ancestor-or-self of
    the source) they name.  Every entry of the result should be 1."""
    parent = np.asarray(parent)
    nb = len(parent)
    anc = []
    for b in range(nb):
        chain, a = [], b
        while a >= 0:
            chain.append(a)
            a = parent[a]
        anc.append(chain)
    leaves = [b for b in range(nb) if role[b] == LEAF]
    out = {}
    for t in leaves:
        mult = {}
        for s in U[t]:
            mult[s] = mult.get(s, 0) + 1
        for s in W[t]:
            mult[s] = mult.get(s, 0) + 1
        for a in anc[t]:
            for s in V[a]:
                mult[s] = mult.get(s, 0) + 1
            for s in X[a]:
                mult[s] = mult.get(s, 0) + 1
        for s in leaves:
            if inst[s] != inst[t]:
                continue
            out[(t, s)] = sum(mult.get(b, 0) for b in anc[s])
    return out


def uniform_tree(xy, D, L):
    """Non-empty boxes of levels 0..L of the quadtree over [0, 2^D)^2 (points relative to
    the root corner), in level order then Morton order: level, x, y, parent, count."""
    xy = np.asarray(xy, dtype=np.int64)
    level, bx, by, par, cnt = [], [], [], [], []
    index = {}
    for lev in range(L + 1):
        sh = D - lev
        cells, counts = np.unique(np.stack([xy[:, 0] >> sh, xy[:, 1] >> sh], axis=1), axis=0, return_counts=True)
        for (cx, cy), c in zip(cells.tolist(), counts.tolist()):
            index[(lev, cx, cy)] = len(level)
            level.append(lev)
            bx.append(cx)
            by.append(cy)
            par.append(index[(lev - 1, cx >> 1, cy >> 1)] if lev > 0 else -1)
            cnt.append(c)
    return (np.array(level), np.array(bx), np.array(by), np.array(par), np.array(cnt))
