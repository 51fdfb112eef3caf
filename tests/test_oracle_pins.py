"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's formulas and compares it with itself:
each checks a closed form, a conservation law, an analytic profile, a
definition evaluated by brute force with a different algorithm, an exact
symmetry, or the values printed in the paper.
"""
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial.distance import pdist

from paper_1112_4539_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Eq. (1) pins
def _closed_pair(xi, xj, mj, eps):
    """Exact two-body term of Eq. (1) in 60-digit decimal arithmetic."""
    getcontext().prec = 60
    d = [Fraction(b) - Fraction(a) for a, b in zip(xi, xj)]
    r2 = sum(x * x for x in d) + Fraction(eps) ** 2
    r = (Decimal(r2.numerator) / Decimal(r2.denominator)).sqrt()
    m = Decimal(Fraction(mj).numerator) / Decimal(Fraction(mj).denominator)
    acc = [m * (Decimal(x.numerator) / Decimal(x.denominator)) / (r * r * r) for x in d]
    pot = -m / r
    return [float(a) for a in acc], float(pot)


@pytest.mark.parametrize("xi,xj,m,eps", [
    ((0.0, 0.0, 0.0), (1.0, 2.0, 2.0), 0.75, 4.0),          # r^2 + eps^2 = 25
    ((0.0, 0.0, 0.0), (3.0, 4.0, 0.0), 2.0, 0.0),           # r = 5, no softening
    ((0.1, -0.2, 0.3), (-0.7, 0.05, 1.9), 0.3, 0.01),
    ((1e3, 1e3, 1e3), (1e3 + 1e-3, 1e3, 1e3 - 2e-3), 1e-6, 0.0),
    ((-5.0, 2.0, 0.5), (4.0, -3.0, 0.25), 7.0, 3.0),
])
def test_two_body_closed_form(oracle_mod, xi, xj, m, eps):
    pos = np.array([xi, xj], np.float64)
    mass = np.array([1.25, m])
    acc, pot, _ = oracle_mod.direct(pos, mass, eps)
    a_ref, p_ref = _closed_pair(xi, xj, m, eps)
    for k in range(3):
        assert abs(acc[0, k] - a_ref[k]) <= 2 * np.spacing(abs(a_ref[k]) + 1e-300)
    assert abs(pot[0] - p_ref) <= 2 * np.spacing(abs(p_ref))
    # the partner feels the opposite pull, scaled by the masses (attractive: toward the source)
    a2, p2 = _closed_pair(xj, xi, 1.25, eps)
    for k in range(3):
        assert abs(acc[1, k] - a2[k]) <= 2 * np.spacing(abs(a2[k]) + 1e-300)
        assert np.sign(acc[0, k]) == np.sign(xj[k] - xi[k]) or xj[k] == xi[k]


def test_exact_two_body_values(oracle_mod):
    # dx = (1,2,2), eps = 4: (r^2+eps^2)^(1/2) = 5 exactly.
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    acc, pot, _ = oracle_mod.direct(pos, np.array([1.0, 0.75]), 4.0)
    np.testing.assert_allclose(acc[0], 0.75 * np.array([1, 2, 2]) / 125.0, rtol=4 * 2.0 ** -52)
    assert abs(pot[0] + 0.15) <= 2 * np.spacing(0.15)


def test_coincident_pairs(oracle_mod):
    pos = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    mass = np.array([2.0, 3.0])
    acc, pot, _ = oracle_mod.direct(pos, mass, 0.25)
    assert np.all(acc == 0.0)
    assert pot[0] == -3.0 / 0.25 and pot[1] == -2.0 / 0.25
    acc, pot, _ = oracle_mod.direct(pos, mass, 0.0)       # unsoftened: pair skipped
    assert np.all(acc == 0.0) and np.all(pot == 0.0)


def test_momentum_conservation_and_pair_energy(oracle_mod):
    rng = np.random.default_rng(11)
    pos = rng.normal(size=(500, 3))
    mass = rng.random(500) + 0.1
    eps = 0.05
    acc, pot, _ = oracle_mod.direct(pos, mass, eps)
    p = (mass[:, None] * acc).sum(0)
    assert np.linalg.norm(p) <= 1e-13 * (mass * np.linalg.norm(acc, axis=1)).sum()
    # sum_i m_i phi_i = 2 W, W = -sum_{i<j} m_i m_j / sqrt(r_ij^2 + eps^2)
    d = pdist(pos)
    mm = pdist(mass[:, None], lambda u, v: u[0] * v[0])
    W = -np.sum(mm / np.sqrt(d * d + eps * eps))
    assert abs(0.5 * (mass * pot).sum() - W) <= 1e-12 * abs(W)


# ----------------------------------------------------- analytic Plummer profile
R_TRUNC = 10.0
M_R = R_TRUNC ** 3 / (1 + R_TRUNC ** 2) ** 1.5


def _phi_t(r):
    return (-(1 + r * r) ** -0.5 + (1 + R_TRUNC ** 2) ** -1.5) / M_R


def _ar_t(r):
    return r * (1 + r * r) ** -1.5 / M_R


def test_plummer_analytic_profile(oracle_mod):
    """Direct sum on the 4096-particle Plummer sphere vs the truncated closed form.

    Radial-bin means; tolerances are a few times the seed-to-seed scatter of
    a 4096-particle realisation (potential ~0.5%, outer acceleration ~1%).
    """
    pos, mass = inputs.plummer(4096, 0)
    acc, pot, _ = oracle_mod.direct(pos, mass, 0.01)
    r = np.linalg.norm(pos, axis=1)
    ar = -(acc * pos).sum(1) / r          # inward radial component
    edges = np.array([0, 0.25, 0.5, 0.75, 1, 1.5, 2, 3, 5, 10.0])
    b = np.digitize(r, edges) - 1
    for k in range(len(edges) - 1):
        s = b == k
        assert abs(pot[s].mean() / _phi_t(r[s]).mean() - 1) < 0.03
        if edges[k] >= 1.0:
            assert abs(ar[s].mean() / _ar_t(r[s]).mean() - 1) < 0.04
    # total energy W = 1/2 sum m phi vs 1/2 int rho phi dV
    rho = lambda x: 3 / (4 * np.pi) * (1 + x * x) ** -2.5 / M_R
    Wa = 0.5 * integrate.quad(lambda x: 4 * np.pi * x * x * rho(x) * _phi_t(x), 0, R_TRUNC,
                              epsabs=1e-13)[0]
    assert abs(0.5 * (mass * pot).sum() / Wa - 1) < 0.02


# ---------------------------------------------------- tree from its definition
def _grid(pos):
    lo = pos.min(0)
    L = (pos.max(0) - lo).max()
    L = 1.0 if L == 0 else L
    q = np.clip(np.floor((pos - lo) * (2.0 ** 21 / L)), 0, 2 ** 21 - 1).astype(np.int64)
    return lo, L, q


def _definition_nodes(pos):
    """Node set of the compressed oct-tree by brute-force enumeration of cells.

    A cell (level k, integer coordinates) is an internal node iff its particles
    occupy at least two of its eight sub-cells.  A one-particle sub-cell of an
    internal node is a leaf; a group of particles that never separates down to
    the finest grid is a bucket leaf at level 21.
    """
    n = len(pos)
    _, _, q = _grid(pos)
    cells = {}
    for k in range(22):
        pref = q >> (21 - k)
        g = {}
        for i in range(n):
            g.setdefault(tuple(int(v) for v in pref[i]), []).append(i)
        cells[k] = g
    internal = set()
    for k in range(21):
        for key, mem in cells[k].items():
            if len({tuple(int(v) for v in (q[i] >> (20 - k))) for i in mem}) >= 2:
                internal.add((k, key))
    leaves = {}
    if n == 1:
        leaves[(0, (0, 0, 0))] = 1
    for (k, key) in internal:
        for ckey, mem in cells[k + 1].items():
            if tuple(v >> 1 for v in ckey) != key:
                continue
            if len(mem) == 1:
                leaves[(k + 1, ckey)] = 1
            elif not any((kk, tuple(int(v) for v in (q[mem[0]] >> (21 - kk)))) in internal
                         for kk in range(k + 1, 21)):
                leaves[(21, tuple(int(v) for v in q[mem[0]]))] = len(mem)
    if not internal and n >= 2:                       # every key identical
        leaves[(21, tuple(int(v) for v in q[0]))] = n
    return internal, leaves


def _morton_perm(pos):
    _, _, q = _grid(pos)
    keys = []
    for i in range(len(pos)):
        k = 0
        for b in range(20, -1, -1):
            k = (k << 3) | (int(q[i, 0] >> b) & 1) << 2 | (int(q[i, 1] >> b) & 1) << 1 | (int(q[i, 2] >> b) & 1)
        keys.append((k, i))
    return np.array([i for _, i in sorted(keys)], np.int64)


def _tree_cases():
    rng = np.random.default_rng(5)
    cases = []
    for n in (1, 2, 3, 5, 8, 13, 16):
        cases.append(rng.random((n, 3)))
    p = rng.random((12, 3))
    p[5] = p[2]; p[9] = p[2]; p[7] = p[1]                  # exact duplicates
    cases.append(p)
    cases.append(np.tile(rng.random((1, 3)), (6, 1)))      # all coincident
    p = rng.random((10, 3))
    p[3] = p[4] + 1e-9                                     # same finest cell, distinct points
    cases.append(p)
    p = np.zeros((9, 3)); p[:, 0] = np.arange(9) * 2.0 ** -18   # collinear, deep split
    cases.append(p)
    return cases


@pytest.mark.parametrize("case", range(len(_tree_cases())))
def test_tree_matches_definition(oracle_mod, case):
    pos = _tree_cases()[case]
    n = len(pos)
    mass = np.random.default_rng(case).random(n) + 0.5
    T = oracle_mod.Tree(pos, mass)
    internal, leaves = _definition_nodes(pos)
    got_int = {(int(T.level[c]), tuple(int(v) for v in T.cell[c])) for c in range(T.n_nodes) if not T.leaf[c]}
    got_leaf = {(int(T.level[c]), tuple(int(v) for v in T.cell[c])): int(T.count[c])
                for c in range(T.n_nodes) if T.leaf[c]}
    assert got_int == internal
    assert got_leaf == leaves
    assert T.n_nodes == len(internal) + len(leaves)
    # Morton order = depth-first leaf order (Sec. 5), ties by input index
    np.testing.assert_array_equal(T.perm, _morton_perm(pos))
    # preorder structure: first child c+1, siblings by next, octant order, counts add up
    for c in range(T.n_nodes):
        assert c < T.next[c] <= T.n_nodes
        if T.leaf[c]:
            assert T.next[c] == c + 1
            continue
        ch, kids = c + 1, []
        while ch < T.next[c]:
            kids.append(ch)
            ch = T.next[ch]
        assert ch == T.next[c] and len(kids) >= 2
        assert sum(int(T.count[k]) for k in kids) == T.count[c]
        octs = []
        for k in kids:
            up = T.cell[k] >> (T.level[k] - T.level[c] - 1)
            assert np.array_equal(up >> 1, T.cell[c])
            octs.append(int(up[0] & 1) * 4 + int(up[1] & 1) * 2 + int(up[2] & 1))
        assert octs == sorted(octs) and len(set(octs)) == len(octs)


def test_moments_and_cell_geometry(oracle_mod):
    pos, mass = inputs.plummer(3000, 7)
    mass = mass * (1 + np.random.default_rng(1).random(3000))
    T = oracle_mod.Tree(pos, mass)
    assert abs(T.M[0] - math.fsum(mass)) <= 1e-15 * T.M[0] * 4
    for d in range(3):
        ref = math.fsum(mass * pos[:, d]) / math.fsum(mass)
        assert abs(T.com[0, d] - ref) <= 1e-14 * max(1.0, abs(ref))
    lo, L, _ = _grid(pos)
    np.testing.assert_array_equal(T.lo, lo)
    assert T.L == L
    for c in range(T.n_nodes):
        assert T.l[c] == L / 2.0 ** T.level[c]
        if T.leaf[c]:
            continue
        kids, ch = [], c + 1
        while ch < T.next[c]:
            kids.append(ch)
            ch = T.next[ch]
        assert abs(sum(T.M[k] for k in kids) - T.M[c]) <= 1e-15 * T.M[c] * len(kids)
        ctr = lo + (T.cell[c] + 0.5) * T.l[c]
        s_ref = float(np.linalg.norm(ctr - T.com[c]))
        assert abs(T.s[c] - s_ref) <= 4e-16 * max(s_ref, 1e-300) + 1e-300
        # the centre of mass lies inside the cell
        assert np.all(T.com[c] >= lo + T.cell[c] * T.l[c] - 1e-12 * L)
        assert np.all(T.com[c] <= lo + (T.cell[c] + 1) * T.l[c] + 1e-12 * L)


# ------------------------------------------------------------------ walk pins
def test_walk_theta_to_zero_is_direct(oracle_mod):
    pos, mass = inputs.plummer(2000, 3)
    T = oracle_mod.Tree(pos, mass)
    w = T.walk(1e-6, 0.01)
    acc, pot, amag = oracle_mod.direct(pos, mass, 0.01)
    assert np.all(w["n_pp"] == 1999) and np.all(w["n_pc"] == 0)
    err = np.linalg.norm(w["acc"] - acc, axis=1) / amag
    assert err.max() < 1e-14
    assert np.max(np.abs(w["pot"] - pot) / np.abs(pot)) < 1e-14


def _expected_lists(T, pos, theta):
    """Interaction set of every particle from the node arrays, by ancestor tests.

    Node c is a cell term of particle i iff i is outside c, c passes the
    opening test, and every proper ancestor of c was opened for i (i inside
    it, or the test failed).  Particle j != i is a particle term iff every
    proper ancestor of j's leaf was opened.
    """
    n, m = T.n, T.n_nodes
    parent = np.full(m, -1)
    for c in range(m):
        if not T.leaf[c]:
            ch = c + 1
            while ch < T.next[c]:
                parent[ch] = c
                ch = T.next[ch]
    rank = np.empty(n, np.int64)
    rank[T.perm] = np.arange(n)
    leaf_of = np.empty(n, np.int64)
    for c in range(m):
        if T.leaf[c]:
            leaf_of[T.perm[T.first[c]:T.first[c] + T.count[c]]] = c
    out = []
    for i in range(n):
        inside = (rank[i] >= T.first) & (rank[i] < T.first + T.count)
        d2 = ((T.com - pos[i]) ** 2).sum(1)
        S = (T.l / theta + T.s) ** 2
        opened = inside | ~(d2 > S)
        opened[T.leaf.astype(bool)] = True
        ok = np.ones(m, bool)             # all proper ancestors opened
        for c in range(m):                # preorder: parents first
            p = parent[c]
            ok[c] = p < 0 or (ok[p] and opened[p])
        words = set()
        for c in range(m):
            if ok[c] and not T.leaf[c] and not opened[c]:
                words.add((c << 1) | 1)
        for j in range(n):
            if j != i and ok[leaf_of[j]]:
                words.add(j << 1)
        out.append(words)
    return out, leaf_of


def test_walk_lists_match_ancestor_definition(oracle_mod):
    pos, mass = inputs.plummer(300, 4)
    T = oracle_mod.Tree(pos, mass)
    theta = 0.7
    w = T.walk(theta, 0.01, maxlen=400)
    exp, leaf_of = _expected_lists(T, pos, theta)
    rank = np.empty(T.n, np.int64)
    rank[T.perm] = np.arange(T.n)
    for i in range(T.n):
        L = int(w["n_pp"][i] + w["n_pc"][i])
        words = [int(x) for x in w["lists"][i, :L]]
        assert set(words) == exp[i] and len(words) == len(exp[i])
        # the walk order is depth-first preorder of the visited nodes
        order = [(x >> 1) if (x & 1) else int(leaf_of[x >> 1]) for x in words]
        assert order == sorted(order)
        # a cell holding i is never used as a cell term
        for x in words:
            if x & 1:
                c = x >> 1
                assert not (T.first[c] <= rank[i] < T.first[c] + T.count[c])
        # the hash summarises the ordered list (FNV-1a over 64-bit words)
        h = 14695981039346656037
        for x in words:
            h = ((h ^ x) * 1099511628211) & (2 ** 64 - 1)
        assert int(w["hash"][i]) == h


def test_walk_permutation_invariance_bitexact(oracle_mod):
    pos, mass = inputs.plummer(3000, 9)
    perm = np.random.default_rng(2).permutation(3000)
    T1 = oracle_mod.Tree(pos, mass)
    T2 = oracle_mod.Tree(pos[perm], mass[perm])
    w1 = T1.walk(0.6, 0.01)
    w2 = T2.walk(0.6, 0.01)
    np.testing.assert_array_equal(w2["acc"], w1["acc"][perm])
    np.testing.assert_array_equal(w2["pot"], w1["pot"][perm])


def test_walk_power_of_two_scaling_bitexact(oracle_mod):
    pos, mass = inputs.plummer(3000, 10)
    w1 = oracle_mod.Tree(pos, mass).walk(0.5, 0.01)
    w2 = oracle_mod.Tree(pos * 2.0, mass * 8.0).walk(0.5, 0.02)
    np.testing.assert_array_equal(w2["acc"], 2.0 * w1["acc"])
    np.testing.assert_array_equal(w2["pot"], 4.0 * w1["pot"])
    np.testing.assert_array_equal(w2["hash"], w1["hash"])


def test_walk_error_vs_theta_and_paper_table(oracle_mod):
    """Error grows with theta like a power ~2-3 (monopole), and at N = 10240 it
    sits within a factor 3 of the paper's printed N=10K column (Sec. 5 table of
    a_error; different particle model, so magnitude only)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "paper_err_a.txt"))
    n = 10240
    pos, mass = inputs.plummer(n, 12)
    T = oracle_mod.Tree(pos, mass)
    tg = inputs.sample_targets(n, 2048, 12)
    acc, _, _ = oracle_mod.direct(pos, mass, 0.01, targets=tg)
    errs = []
    for theta, paper10k in zip(tab[:, 0], tab[:, 1]):
        w = T.walk(theta, 0.01, targets=tg)
        e = oracle_mod.mean_rel_err(w["acc"], acc)
        errs.append(e)
        assert paper10k / 3 < e < paper10k * 3, (theta, e, paper10k)
    assert all(b > a for a, b in zip(errs, errs[1:]))
    slope = np.polyfit(np.log(tab[:, 0]), np.log(errs), 1)[0]
    assert 1.5 < slope < 3.5


# ------------------------------------------ A_i = sum_j |f_ij| (cancellation floor)
def test_amag_two_body_equals_force(oracle_mod):
    # one term: the sum of term magnitudes is the force itself, |a| = m r / (r^2 + eps^2)^(3/2)
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    acc, _, amag = oracle_mod.direct(pos, np.array([1.0, 0.75]), 4.0)
    assert abs(amag[0] - 0.75 * 3.0 / 125.0) <= 4 * np.spacing(0.018)
    assert abs(amag[1] - 1.0 * 3.0 / 125.0) <= 4 * np.spacing(0.024)
    np.testing.assert_allclose(amag, np.linalg.norm(acc, axis=1), rtol=4e-16)


def test_amag_collinear_sources_equals_force(oracle_mod):
    # every source on the +x ray from the target: all terms point the same way, so
    # sum |f| = |sum f|, while a term that forgot |dx| or used the softened distance would not match
    xs = np.array([0.0, 0.3, 1.0, 2.5, 4.0, 7.25])
    pos = np.zeros((len(xs), 3))
    pos[:, 0] = xs
    mass = np.array([1.0, 0.5, 2.0, 0.25, 3.0, 1.5])
    eps = 0.2
    acc, _, amag = oracle_mod.direct(pos, mass, eps, targets=np.array([0]))
    ref = math.fsum(float(m) * float(x) / (float(x) ** 2 + eps * eps) ** 1.5 for m, x in zip(mass[1:], xs[1:]))
    assert abs(amag[0] - ref) <= 1e-15 * ref
    assert abs(acc[0, 0] - ref) <= 1e-15 * ref and acc[0, 1] == 0.0 and acc[0, 2] == 0.0


def test_amag_symmetric_pair_cancels(oracle_mod):
    # sources at +-r e_x: the force cancels exactly, A = 2 m r / (r^2 + eps^2)^(3/2)
    r, m, eps = 0.75, 0.4, 0.5
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0], [-r, 0.0, 0.0]])
    acc, _, amag = oracle_mod.direct(pos, np.array([1.0, m, m]), eps, targets=np.array([0]))
    assert np.all(acc[0] == 0.0)
    _, p = _closed_pair((0.0, 0.0, 0.0), (r, 0.0, 0.0), m, eps)   # p = -m / sqrt(r^2 + eps^2)
    ref = 2.0 * (-p) * r / (r * r + eps * eps)
    assert abs(amag[0] - ref) <= 4 * np.spacing(ref)


def test_amag_of_walk_cell_and_limit(oracle_mod):
    # theta -> 0: the walk's A equals the direct sum's (same terms, another order)
    pos, mass = inputs.plummer(1500, 13)
    w = oracle_mod.Tree(pos, mass).walk(1e-6, 0.01)
    _, _, amag = oracle_mod.direct(pos, mass, 0.01)
    np.testing.assert_allclose(w["amag"], amag, rtol=1e-13)
    # a far target sees a compact cluster as one cell term: A = M d / (d^2 + eps^2)^(3/2), d to the
    # cluster's centre of mass
    rng = np.random.default_rng(3)
    cl = rng.random((50, 3)) * 1e-3
    pos = np.vstack([cl, [[10.0, 0.0, 0.0]]])
    mass = np.full(51, 0.02)
    T = oracle_mod.Tree(pos, mass)
    w = T.walk(0.5, 0.05, targets=np.array([50]))
    assert w["n_pc"][0] == 1 and w["n_pp"][0] == 0
    com = (mass[:50, None] * cl).sum(0) / mass[:50].sum()
    d = np.linalg.norm(com - pos[50])
    assert abs(w["amag"][0] - 1.0 * d / (d * d + 0.05 ** 2) ** 1.5) <= 1e-12
