"""Pins of the oracle's Hilbert walk order (oracle/hilbert.py) by the defining properties of the
curve (Sec. 5, the Peano-Hilbert ordering), independent of the GPU."""
import numpy as np
import pytest

from oracle import hilbert
from paper_1112_4539_amd import inputs


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5])
def test_hilbert_index_is_a_face_connected_bijection(b):
    s = 1 << b
    g = np.stack(np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij"), -1).reshape(-1, 3)
    h = hilbert_index = hilbert.hilbert_index(g, b)
    # a bijection of the 8^b cells onto [0, 8^b)
    assert np.array_equal(np.sort(h), np.arange(s ** 3))
    cells = np.empty((s ** 3, 3), np.int64)
    cells[h] = g
    # consecutive cells share a face: one coordinate differs by one
    d = np.abs(np.diff(cells, axis=0))
    assert np.all(d.sum(1) == 1)
    # starts at the origin; the b-bit curve restricted to its first 8^(b-1) cells is the lower octant
    assert tuple(cells[0]) == (0, 0, 0)
    if b > 1:
        assert np.all(cells[: s ** 3 // 8] < s // 2)
    del hilbert_index


def test_hilbert_index_nested_levels():
    # the index of a cell at b levels, shifted down by 3, is the index of its parent at b - 1
    rng = np.random.default_rng(0)
    q = rng.integers(0, 1 << 10, (5000, 3))
    assert np.array_equal(hilbert.hilbert_index(q, 10) >> 3, hilbert.hilbert_index(q >> 1, 9))


def test_walk_order_permutation_and_ties():
    pos, mass = inputs.clumpy(20_000, 7)
    pos = pos.astype(np.float32).astype(np.float64)
    # duplicates: 500 particles copied onto others (ties in the Hilbert key keep Morton order)
    pos[-500:] = pos[:500]
    o = hilbert.walk_order(pos, mass)
    assert np.array_equal(np.sort(o), np.arange(len(pos)))
    # the order follows the curve: the level-10 Hilbert index never decreases along it, and
    # neighbours along it lie in the same or face-adjacent level-4 cells (a few particles per
    # cell) far more often than along a random order
    from oracle import Tree
    T = Tree(pos, mass)
    g = hilbert._grid(pos, T)
    assert np.all(np.diff(hilbert.hilbert_index(g[o] >> 11, 10)) >= 0)
    q = g >> 17
    adj = np.abs(np.diff(q[o], axis=0)).sum(1) <= 1
    rnd = np.abs(np.diff(q[np.random.default_rng(1).permutation(len(pos))], axis=0)).sum(1) <= 1
    assert adj.mean() > 0.8 and adj.mean() > 5 * rnd.mean()
    # ties: particles with equal keys keep their Morton (tree) order
    rank = np.empty(len(pos), np.int64)
    rank[T.perm] = np.arange(len(pos))
    h = hilbert.hilbert_index(g[o] >> 11, 10)
    same = h[1:] == h[:-1]
    assert same.any() and np.all(rank[o][1:][same] > rank[o][:-1][same])


def test_walk_order_forest_clusters_contiguous():
    rng = np.random.default_rng(3)
    sizes = [300, 1, 0, 2000, 77]
    off = np.concatenate([[0], np.cumsum(sizes)])
    pos = rng.random((off[-1], 3))
    mass = np.ones(off[-1])
    o = hilbert.walk_order(pos, mass, off)
    assert np.array_equal(np.sort(o), np.arange(off[-1]))
    cl = np.searchsorted(off, o, side="right") - 1
    assert np.all(np.diff(cl) >= 0)
    assert hilbert.levels_for(5) == 9 and hilbert.levels_for(1) == 10 and hilbert.levels_for(1 << 24) == 5
