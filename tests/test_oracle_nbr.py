"""Pins of the oracle's neighbour search (the general tree walk of Sec. 4.3, Fig. 4)
and of its per-neighbour work, the SPH density sum.

The walk's neighbour sets are checked against brute force over all pairs and
against scipy's k-d tree; the density against the brute-force sum, a lattice
whose density is known, and the kernel's normalisation.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

from paper_1112_4539_amd import inputs
from tests.util import tree_cases


@pytest.mark.parametrize("h", [0.3, 1.0, 2.5])
def test_sph_kernel_normalised_and_continuous(oracle_mod, h):
    W = lambda r: oracle_mod.sph_kernel(r, h)
    total = integrate.quad(lambda r: 4 * np.pi * r * r * W(r), 0, 2 * h, points=[h], epsabs=1e-14)[0]
    assert abs(total - 1.0) < 1e-12
    assert W(0.0) == pytest.approx(1.0 / (np.pi * h ** 3), rel=1e-15)
    for q in (1.0, 2.0):                       # continuous where the pieces meet
        assert abs(W(q * h * (1 - 1e-12)) - W(q * h)) < 1e-9 * W(0.0)
    assert W(2.0 * h) == 0.0 and W(3.0 * h) == 0.0


def _sets(lists, counts):
    return [set(int(x) for x in row[:c]) for row, c in zip(lists, counts)]


@pytest.mark.parametrize("case,radius", [("random1000", 0.08), ("random1000", 0.3), ("duplicates", 0.5),
                                         ("coincident", 0.1), ("finest_cell_pair", 0.2), ("flat", 0.01),
                                         ("collinear_deep", 2.0 ** -17)])
def test_neighbours_against_brute_force_and_kdtree(oracle_mod, case, radius):
    pos = tree_cases()[case]
    n = len(pos)
    mass = np.random.default_rng(n).random(n) + 0.5
    T = oracle_mod.Tree(pos, mass)
    out = T.neighbours(radius, maxlen=n)
    cnt, rho = oracle_mod.neighbours_brute(pos, mass, radius)
    np.testing.assert_array_equal(out["count"], cnt)
    np.testing.assert_allclose(out["rho"], rho, rtol=1e-13)
    kd = cKDTree(pos)
    got = _sets(out["lists"], out["count"])
    for i in range(n):
        want = {j for j in kd.query_ball_point(pos[i], radius) if j != i
                and np.sum((pos[j] - pos[i]) ** 2) < radius * radius}
        assert got[i] == want, i
    # lists in the walk's order (depth-first: ascending Morton position) and their hash
    rank = np.empty(n, np.int64)
    rank[T.perm] = np.arange(n)
    for i in range(n):
        row = [int(x) for x in out["lists"][i, :out["count"][i]]]
        assert [rank[j] for j in row] == sorted(rank[j] for j in row)
        h = 14695981039346656037
        for j in row:
            h = ((h ^ (j << 1)) * 1099511628211) & (2 ** 64 - 1)
        assert int(out["hash"][i]) == h


def test_neighbours_clumpy_sampled(oracle_mod):
    pos, mass = inputs.clumpy(40_000, 17)
    T = oracle_mod.Tree(pos, mass)
    tg = inputs.sample_targets(len(pos), 500, 3)
    out = T.neighbours(0.01, targets=tg)
    cnt, rho = oracle_mod.neighbours_brute(pos, mass, 0.01, targets=tg)
    np.testing.assert_array_equal(out["count"], cnt)
    np.testing.assert_allclose(out["rho"], rho, rtol=1e-13)
    assert cnt.max() > 100 and cnt.min() >= 0


def test_density_of_a_lattice(oracle_mod):
    """A cubic lattice of spacing a with masses a^3 has density 1; the M4 sum with h = 1.2 a
    (support 2.4 a: no lattice point at the edge of the ball) reproduces it to 0.1 percent away
    from the lattice's edges."""
    k = 20
    a = 1.0 / k
    g = (np.arange(k) + 0.5) * a
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    mass = np.full(len(pos), a ** 3)
    h = 1.2 * a
    T = oracle_mod.Tree(pos, mass)
    inner = np.where(np.all((pos > 2 * h + 1e-9) & (pos < 1 - 2 * h - 1e-9), axis=1))[0]
    out = T.neighbours(2 * h, targets=inner)
    assert np.all(np.abs(out["rho"] - 1.0) < 1e-3)
    assert np.all(out["count"] == out["count"][0])     # every interior particle sees the same shell
