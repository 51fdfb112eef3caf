"""Hilbert walk order of the targets -- TEST INFRASTRUCTURE (see the package header).

Sec. 5 notes that a Peano-Hilbert ordering of the particles localizes a walk
further than the Morton order.  The walk runs its targets in groups of 64
consecutive entries of an order; this module gives that order:

* ``hilbert_index(q, b)``: index of cell q = (x, y, z) of a 2^b grid along
  the three-dimensional Hilbert curve, by Skilling's transform (J. Skilling,
  "Programming the Hilbert curve", AIP Conf. Proc. 707, 381 (2004)): undo the
  excess work of the Gray-code traversal level by level (invert or exchange
  the low bits against the first axis), Gray-encode across the axes, then
  read the bits out with x the most significant of each triplet.
* ``walk_order(pos, clusters=None)``: the targets (caller indices) sorted by
  (cluster, Hilbert index of the cell `levels` levels below the cluster's
  root cube), ties in Morton order.  The cell of a particle is taken from its
  coordinates on the 2^21 grid of its cluster's root cube, the grid of the
  Morton keys (Sec. 4.1); `levels` is 10 for one tree, and for a forest of K
  clusters max(5, min(10, (32 - bits(K - 1)) // 3)).

Plain numpy, vectorised over the particles; the tree (Morton order) comes from
the oracle's own build.
"""
from __future__ import annotations

import numpy as np

GRID_BITS = 21


def hilbert_index(q, b):
    """Hilbert index (int64) of the cells q [n, 3] (integers in [0, 2^b)) of a 2^b grid."""
    X = [np.asarray(q[:, i], dtype=np.int64).copy() for i in range(3)]
    if b <= 0:
        return np.zeros(len(X[0]), np.int64)
    Q = 1 << (b - 1)
    while Q > 1:
        P = Q - 1
        for i in range(3):
            hit = (X[i] & Q) != 0
            # bit set: invert the low bits of the first axis
            X[0] = np.where(hit, X[0] ^ P, X[0])
            # bit clear: exchange the low bits of the first axis and axis i
            t = np.where(hit, 0, (X[0] ^ X[i]) & P)
            X[0] = X[0] ^ t
            X[i] = X[i] ^ t
        Q >>= 1
    X[1] = X[1] ^ X[0]
    X[2] = X[2] ^ X[1]
    t = np.zeros_like(X[0])
    Q = 1 << (b - 1)
    while Q > 1:
        t = np.where((X[2] & Q) != 0, t ^ (Q - 1), t)
        Q >>= 1
    X = [x ^ t for x in X]
    h = np.zeros_like(X[0])
    for j in range(b - 1, -1, -1):
        for i in range(3):
            h = (h << 1) | ((X[i] >> j) & 1)
    return h


def levels_for(n_clusters):
    cbits = int(n_clusters - 1).bit_length()
    return max(5, min(10, (32 - cbits) // 3))


def _grid(pos, tree):
    """Coordinates of the particles on the 2^21 grid of the tree's root cube (as the build
    computes them: floor((x - lo) 2^21 / L), clamped to the grid)."""
    scale = float(1 << GRID_BITS) / tree.L
    g = np.floor((np.asarray(pos, np.float64) - tree.lo[None, :]) * scale)
    return np.clip(g, 0, (1 << GRID_BITS) - 1).astype(np.int64)


def walk_order(pos, mass, offsets=None):
    """Caller indices in walk order for the particles pos [n, 3], mass [n] (float64; one tree, or
    a forest of clusters [offsets[k], offsets[k+1]), each its own tree)."""
    from oracle import Tree
    pos = np.asarray(pos, np.float64)
    mass = np.asarray(mass, np.float64)
    n = len(pos)
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    offsets = np.asarray(offsets, np.int64)
    K = len(offsets) - 1
    b = levels_for(K)
    out = []
    for k in range(K):
        a, e = int(offsets[k]), int(offsets[k + 1])
        if e <= a:
            continue
        T = Tree(pos[a:e], mass[a:e])
        q = _grid(pos[a:e], T) >> (GRID_BITS - b)
        h = hilbert_index(q, b)
        # Morton positions of this cluster sorted by the Hilbert index, ties in Morton order
        mp = np.argsort(h[T.perm], kind="stable")
        out.append(a + T.perm[mp])
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def walk_positions(pos, mass):
    """Morton positions (of the oracle's tree of pos, mass) in walk order, for one tree."""
    from oracle import Tree
    T = Tree(np.asarray(pos, np.float64), np.asarray(mass, np.float64))
    rank = np.empty(T.n, np.int64)
    rank[T.perm] = np.arange(T.n)
    return rank[walk_order(pos, mass)]
