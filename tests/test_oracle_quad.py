"""Pins of the oracle's quadrupole cell term (order 2).

The paper allows any higher moment in the particle-cell term (Sec. 4.1) and
names higher multipoles as the next step (Sec. 7).  The oracle's order-2 term
is the second-order Taylor expansion of the softened cell potential about the
centre of mass.  These tests check it against things it must agree with and
that do not re-type its formula: closed-form second moments, the parallel-axis
theorem between a cell and its children, the exact sum it approximates (the
remainder must shrink one power faster than the monopole's), the gradient of
its own potential, and the whole walk's accuracy and invariances.
"""
import numpy as np
import pytest

from paper_1112_4539_amd import inputs


def test_second_moments_closed_forms(oracle_mod):
    # two equal masses at c +- y: B = 2 m y y^T about their centre of mass
    c = np.array([0.3, 0.4, 0.5])
    y = np.array([0.01, -0.02, 0.005])
    far = np.array([[5.0, 5.0, 5.0]])
    pos = np.vstack([c + y, c - y, far])
    T = oracle_mod.Tree(pos, np.array([0.75, 0.75, 1.0]))
    B = T.B
    pair = [k for k in range(T.n_nodes) if T.count[k] == 2 and not T.leaf[k]][0]
    want = 2 * 0.75 * np.outer(y, y)
    np.testing.assert_allclose(B[pair], want[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]], rtol=1e-12, atol=1e-20)
    # eight unit masses on the corners of a cube of half-side h: B = 8 h^2 I
    h = 0.125
    corners = np.array([[sx, sy, sz] for sx in (-h, h) for sy in (-h, h) for sz in (-h, h)]) + 0.5
    T = oracle_mod.Tree(corners, np.ones(8))
    np.testing.assert_allclose(T.B[0], [8 * h * h, 0, 0, 8 * h * h, 0, 8 * h * h], atol=1e-15)
    # one-particle leaves carry no second moment
    assert np.all(T.B[T.leaf.astype(bool)] == 0.0)


def test_second_moments_parallel_axis(oracle_mod):
    """Each cell's moments equal its children's, shifted to the parent's centre of mass by the
    parallel-axis theorem (a different route than the oracle's direct sum over particles)."""
    pos, mass = inputs.clumpy(3000, 14)
    mass = mass * (1 + np.random.default_rng(2).random(3000))
    T = oracle_mod.Tree(pos, mass)
    B = T.B
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    checked = 0
    for c in range(T.n_nodes):
        if T.leaf[c]:
            continue
        acc = np.zeros(6)
        ch = c + 1
        while ch < T.next[c]:
            d = T.com[ch] - T.com[c]
            acc += B[ch] + T.M[ch] * np.array([d[a] * d[b] for a, b in idx])
            ch = T.next[ch]
        scale = np.abs(B[c][[0, 3, 5]]).sum()
        np.testing.assert_allclose(acc, B[c], rtol=0, atol=1e-12 * scale + 1e-300)
        checked += 1
    assert checked > 500


def _cell(n, seed, symmetric=False):
    rng = np.random.default_rng(seed)
    y = rng.normal(size=(n, 3)) * np.array([1.0, 0.6, 0.3])
    m = rng.random(n) + 0.5
    if symmetric:                              # pairs at +-y with equal masses: no third moment
        y = np.vstack([y, -y])
        m = np.concatenate([m, m])
    return y, m


def _exact_and_terms(oracle_mod, y, m, s, xt, eps):
    """Exact sum at target xt of the cell scaled by s, and the order-1 and order-2 cell terms."""
    cm = np.array([0.1, -0.2, 0.3])
    pts = cm + s * (y - (m[:, None] * y).sum(0) / m.sum())
    com = (m[:, None] * pts).sum(0) / m.sum()
    yy = pts - com
    B = np.array([(m * yy[:, a] * yy[:, b]).sum() for a, b in [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]])
    allp = np.vstack([xt[None, :], pts])
    acc, pot, _ = oracle_mod.direct(allp, np.concatenate([[1.0], m]), eps, targets=np.array([0]))
    a1, p1 = oracle_mod.cell_term(xt, com, m.sum(), B, eps, order=1)
    a2, p2 = oracle_mod.cell_term(xt, com, m.sum(), B, eps, order=2)
    return acc[0], pot[0], a1, p1, a2, p2


@pytest.mark.parametrize("eps", [0.0, 0.3])
@pytest.mark.parametrize("symmetric", [False, True])
def test_cell_term_remainder_orders(oracle_mod, eps, symmetric):
    """Against the exact sum over the cell's particles, the monopole's error falls as size^2 and
    the quadrupole's as size^3 (size^4 when the cell has no third moment)."""
    y, m = _cell(7, 21, symmetric)
    xt = np.array([2.3, 1.1, -0.7])
    sizes = np.array([0.2, 0.1, 0.05, 0.025])
    e1, e2, q1, q2 = [], [], [], []
    for s in sizes:
        a, p, a1, p1, a2, p2 = _exact_and_terms(oracle_mod, y, m, s, xt, eps)
        e1.append(np.linalg.norm(a1 - a) / np.linalg.norm(a))
        e2.append(np.linalg.norm(a2 - a) / np.linalg.norm(a))
        q1.append(abs(p1 - p) / abs(p))
        q2.append(abs(p2 - p) / abs(p))
    sl = lambda e: np.polyfit(np.log(sizes), np.log(e), 1)[0]
    assert abs(sl(e1) - 2) < 0.15 and abs(sl(q1) - 2) < 0.15
    want = 4 if symmetric else 3
    assert abs(sl(e2) - want) < 0.25, sl(e2)
    assert abs(sl(q2) - want) < 0.25, sl(q2)
    assert all(b < a for a, b in zip(e1, e2))


def test_cell_term_force_is_minus_gradient_of_potential(oracle_mod):
    rng = np.random.default_rng(4)
    com = np.array([0.2, 0.1, -0.3])
    B = np.array([0.02, 0.004, -0.003, 0.011, 0.002, 0.007])
    for eps in (0.0, 0.2):
        xt = com + rng.normal(size=3)
        a, _ = oracle_mod.cell_term(xt, com, 1.7, B, eps, order=2)
        h = 1e-5
        g = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            g[k] = -(oracle_mod.cell_term(xt + e, com, 1.7, B, eps, 2)[1]
                     - oracle_mod.cell_term(xt - e, com, 1.7, B, eps, 2)[1]) / (2 * h)
        np.testing.assert_allclose(a, g, rtol=1e-8)


@pytest.mark.parametrize("which,theta,eps", [("plummer", 0.5, 0.01), ("plummer", 0.75, 0.01),
                                             ("clumpy", 0.6, 1e-4)])
def test_walk_quadrupole_beats_monopole(oracle_mod, which, theta, eps):
    """Same opening test, so the same lists; the quadrupole walk is closer to the direct sum."""
    if which == "plummer":
        pos, mass = inputs.plummer(4096, 0)
    else:
        pos, mass = inputs.clumpy(20_000, 15)
    T = oracle_mod.Tree(pos, mass)
    tg = inputs.sample_targets(len(pos), 1024, 3)
    a_ref, p_ref, _ = oracle_mod.direct(pos, mass, eps, targets=tg)
    w1 = T.walk(theta, eps, targets=tg, order=1)
    w2 = T.walk(theta, eps, targets=tg, order=2)
    np.testing.assert_array_equal(w1["hash"], w2["hash"])
    np.testing.assert_array_equal(w1["n_pc"], w2["n_pc"])
    r1 = oracle_mod.rms_rel_err(w1["acc"], a_ref)
    r2 = oracle_mod.rms_rel_err(w2["acc"], a_ref)
    assert r2 < 0.6 * r1, (r1, r2)
    assert np.sqrt(np.mean(((w2["pot"] - p_ref) / p_ref) ** 2)) < np.sqrt(np.mean(((w1["pot"] - p_ref) / p_ref) ** 2))


def test_walk_quadrupole_limits_and_scaling(oracle_mod):
    pos, mass = inputs.plummer(1500, 17)
    T = oracle_mod.Tree(pos, mass)
    w = T.walk(1e-6, 0.01, order=2)                       # no cell accepted: the direct sum
    acc, pot, amag = oracle_mod.direct(pos, mass, 0.01)
    assert np.all(w["n_pc"] == 0)
    assert (np.linalg.norm(w["acc"] - acc, axis=1) / amag).max() < 1e-14
    w1 = T.walk(0.6, 0.01, order=2)
    w2 = oracle_mod.Tree(pos * 2.0, mass * 8.0).walk(0.6, 0.02, order=2)
    np.testing.assert_array_equal(w2["acc"], 2.0 * w1["acc"])
    np.testing.assert_array_equal(w2["pot"], 4.0 * w1["pot"])
