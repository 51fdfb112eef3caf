"""Pins of the learned-opening-parameter oracle (CPU only).

Each definition is held to something other than itself: torch's bfloat16
conversion and tanh-form GELU (library routines), a torch composition of the
same layers, central finite differences of the loss, torch's Adam, an
analytic lattice for the geometric features, and a brute-force search for the
containing cell.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import learn


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -(1.0 + 2.0 ** -8),
         3.0e38, -3.0e38, 1e-40, -1e-40, 2.0 ** -149, 2.0 ** -126 * (1 + 2.0 ** -8), np.inf, -np.inf],
    ])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = learn.bf16(x32)
    np.testing.assert_array_equal(got, ref)
    # ties go to even
    assert learn.bf16(1.0 + 2.0 ** -8) == 1.0
    assert learn.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert np.isnan(learn.bf16(np.nan))


def test_gelu_matches_torch_and_its_derivative():
    x = np.linspace(-8, 8, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="tanh").numpy()
    np.testing.assert_allclose(learn.gelu(x), ref, rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (learn.gelu(x + h) - learn.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(learn.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def _problem(seed, rows=96):
    rng = np.random.default_rng(seed)
    P = learn.init_params(seed)
    P[learn.LAYOUT["b1"][0]:learn.LAYOUT["b1"][0] + 64] = rng.normal(0, 0.3, 64)
    P[learn.LAYOUT["b2"][0]:learn.LAYOUT["b2"][0] + 64] = rng.normal(0, 0.3, 64)
    P[4800] = 0.2
    X = rng.normal(0, 2, (rows, 8)) + 1.0
    mu = rng.normal(1, 0.1, 8)
    inv_sd = rng.uniform(0.3, 0.7, 8)
    t = rng.uniform(0, 1, rows)
    return P, X, mu, inv_sd, t


def test_forward_matches_torch_layers():
    P, X, mu, inv_sd, _ = _problem(1)
    p = learn.unpack(P)
    net = torch.nn.Sequential(torch.nn.Linear(8, 64), torch.nn.GELU(approximate="tanh"), torch.nn.Linear(64, 64),
                              torch.nn.GELU(approximate="tanh"), torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(p["W1"])); net[0].bias.copy_(torch.from_numpy(p["b1"]))
        net[2].weight.copy_(torch.from_numpy(p["W2"])); net[2].bias.copy_(torch.from_numpy(p["b2"]))
        net[4].weight.copy_(torch.from_numpy(p["w3"][None, :])); net[4].bias.copy_(torch.from_numpy(p["b3"]))
        z = net(torch.from_numpy((X - mu) * inv_sd)).numpy()[:, 0]
    f = learn.forward(P, X, mu, inv_sd, emulate=False)
    np.testing.assert_allclose(f["z"], z, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(f["theta"], 0.2 + 0.8 / (1 + np.exp(-z)), rtol=1e-13)
    # zero weights: theta is the sigmoid of the last bias alone
    P0 = np.zeros(learn.N_PARAM); P0[4800] = -0.7
    np.testing.assert_allclose(learn.forward(P0, X, mu, inv_sd)["theta"], 0.2 + 0.8 / (1 + np.exp(0.7)), rtol=1e-15)


def test_gradient_matches_finite_differences():
    P, X, mu, inv_sd, t = _problem(2)
    _, g = learn.loss_and_grad(P, X, t, mu, inv_sd, emulate=False)
    h = 1e-6
    fd = np.empty_like(P)
    for k in range(len(P)):
        Pp = P.copy(); Pp[k] += h
        Pm = P.copy(); Pm[k] -= h
        fd[k] = (learn.loss_and_grad(Pp, X, t, mu, inv_sd, emulate=False)[0]
                 - learn.loss_and_grad(Pm, X, t, mu, inv_sd, emulate=False)[0]) / (2 * h)
    for name, (o, s) in learn.LAYOUT.items():
        sl = slice(o, o + int(np.prod(s)))
        err = np.linalg.norm(g[sl] - fd[sl]) / np.linalg.norm(g[sl])
        assert err <= 1e-7, (name, err)


def test_rounded_gradient_close_to_exact():
    P, X, mu, inv_sd, t = _problem(3, rows=512)
    l0, g0 = learn.loss_and_grad(P, X, t, mu, inv_sd, emulate=False)
    l1, g1 = learn.loss_and_grad(P, X, t, mu, inv_sd, emulate=True)
    assert abs(l1 - l0) <= 0.02 * l0
    for name, (o, s) in learn.LAYOUT.items():
        sl = slice(o, o + int(np.prod(s)))
        assert np.linalg.norm(g1[sl] - g0[sl]) <= 0.05 * np.linalg.norm(g0[sl]), name


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    P = rng.normal(size=50)
    m = np.zeros(50); v = np.zeros(50)
    w = torch.tensor(P.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=50)
        P, m, v = learn.adam(P, g, m, v, step, 3e-3)
        w.grad = torch.from_numpy(g.copy())
        opt.step()
    np.testing.assert_allclose(P, w.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_lattice():
    """16^3 lattice, equal masses: every Morton group is a 4x4x4 block of the lattice."""
    s = 1.0 / 16
    g = (np.arange(16) + 0.5) * s
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    mass = np.full(len(pos), 1.0 / len(pos))
    T = oracle.Tree(pos, mass)
    X = learn.features(T, pos, mass)
    L = T.L
    h = 1.5 * s
    np.testing.assert_allclose(X[:, 0], np.log2(h / (0.5 * L * (64 / 4096) ** (1 / 3))), rtol=1e-12)
    np.testing.assert_allclose(X[:, 3], np.sqrt(3 * 1.25) * s / h, rtol=1e-12)
    np.testing.assert_allclose(X[:, 4], 0.0, atol=1e-12)


def test_features_cells_brute_force():
    rng = np.random.default_rng(6)
    from paper_1112_4539_amd import inputs
    pos, mass = inputs.plummer(1500, 8)
    mass = mass * rng.uniform(0.5, 1.5, len(mass))
    T = oracle.Tree(pos, mass)
    X = learn.features(T, pos, mass)
    n = len(pos)
    rho_mean = T.M[0] / T.L ** 3
    for g in range((n + 63) // 64):
        a, b = 64 * g, min(n, 64 * g + 64)
        holds = [c for c in range(len(T.M)) if T.first[c] <= a and T.first[c] + T.count[c] >= b]
        c = max(holds, key=lambda k: (T.level[k], k))
        parents = [p for p in holds if p != c and T.first[p] <= T.first[c] and T.next[p] >= T.next[c] and p < c]
        par = max(parents, key=lambda k: T.level[k]) if parents else c
        np.testing.assert_allclose(X[g, 5], np.log10(T.M[c] / T.l[c] ** 3 / rho_mean), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(X[g, 6], np.log10(T.M[par] / T.l[par] ** 3 / rho_mean), rtol=1e-12, atol=1e-12)
        ps = pos[T.perm[a:b]]
        h = max(np.max(ps.max(0) - ps.min(0)) / 2, T.L * 2.0 ** -22)
        np.testing.assert_allclose(X[g, 7], np.log2(T.l[c] / h), rtol=1e-12)
        ancestors = sorted([p for p in holds if p != c], key=lambda k: T.level[k])
        anc = ancestors[-3] if len(ancestors) >= 3 else 0
        w = mass[T.perm[a:b]]
        com = (w[:, None] * ps).sum(0) / w.sum()
        np.testing.assert_allclose(X[g, 1], np.linalg.norm(com - T.com[c]) / T.l[c], rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(X[g, 2], np.linalg.norm(com - T.com[anc]) / T.l[anc], rtol=1e-9, atol=1e-12)


def test_group_rms_definition():
    n = 200
    rng = np.random.default_rng(7)
    ref = rng.normal(size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    acc = ref + 1e-3 * np.linalg.norm(ref, axis=1)[:, None] * d   # relative error exactly 1e-3
    perm = rng.permutation(n)
    r = learn.group_rms(acc, ref, perm)
    assert r.shape == (4,)
    np.testing.assert_allclose(r, 1e-3, rtol=1e-9)


def test_group_rms_skips_zero_reference():
    # a particle with a_ref = 0 has no relative error: left out of its group's mean
    n = 130
    rng = np.random.default_rng(8)
    ref = rng.normal(size=(n, 3))
    acc = ref * (1 + 2e-3)                     # relative error exactly 2e-3 (up to rounding)
    ref[5] = 0.0
    acc[5] = 1.0
    ref[64:128] = 0.0                          # a whole group of zero references
    perm = np.arange(n)
    r = learn.group_rms(acc, ref, perm)
    np.testing.assert_allclose(r[[0, 2]], 2e-3, rtol=1e-9)
    assert r[1] == 0.0 and np.all(np.isfinite(r))


# ------------------------------------------------ label allocation (host, learn.allocate)
def _alloc_tables(seed, K=4, G=6):
    rng = np.random.default_rng(seed)
    # error falls and cost rises toward small theta (grid index 0), with noise
    R = np.sort(rng.uniform(1e-4, 4e-3, (K, G)), axis=0)
    C = np.sort(rng.uniform(10, 200, (K, G)), axis=0)[::-1].copy()
    n_g = rng.integers(1, 65, G).astype(np.float64)
    return R, C, n_g


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("target", [8e-4, 1.5e-3, 2.5e-3])
def test_allocate_against_enumeration(seed, target):
    """learn.allocate picks a Lagrangian point of min C s.t. error <= target: its error is within
    the target, and no choice of grid index per group (all K^G enumerated) with an error no larger
    has a lower total cost."""
    import itertools
    from paper_1112_4539_amd import learn as plearn
    R, C, n_g = _alloc_tables(seed)
    K, G = R.shape
    k = plearn.allocate(R, C, n_g, target)
    N = n_g.sum()
    err = lambda ks: math.sqrt(sum(n_g[g] * R[ks[g], g] ** 2 for g in range(G)) / N)
    cost = lambda ks: sum(C[ks[g], g] for g in range(G))
    e_k, c_k = err(k), cost(k)
    feasible = [ks for ks in itertools.product(range(K), repeat=G) if err(ks) <= target]
    if not feasible:                           # nothing meets the target: the most accurate choice
        assert np.all(k == np.argmin(C + 1e40 * n_g * R * R, axis=0))
        return
    assert e_k <= target * (1 + 1e-12)
    best_at_ek = min(cost(ks) for ks in itertools.product(range(K), repeat=G) if err(ks) <= e_k * (1 + 1e-12))
    assert c_k <= best_at_ek * (1 + 1e-12)


def test_allocate_ignores_non_finite_groups():
    from paper_1112_4539_amd import learn as plearn
    R, C, n_g = _alloc_tables(3, K=5, G=8)
    k0 = plearn.allocate(R, C, n_g, 2e-3)
    R2 = np.hstack([R, np.full((5, 1), np.inf)])
    C2 = np.hstack([C, np.full((5, 1), 50.0)])
    k2 = plearn.allocate(R2, C2, np.append(n_g, 64.0), 2e-3)
    assert k2[-1] == 0
    np.testing.assert_array_equal(k2[:-1], k0)
    # a single non-finite entry is avoided, the rest of its column still usable
    R3 = R.copy()
    R3[4, 2] = np.nan
    k3 = plearn.allocate(R3, C, n_g, 2e-3)
    assert k3[2] != 4 and np.all(k3 >= 0)


def test_features_walk_groups_brute_force():
    """Walk groups of the Hilbert order: members order[64g, 64g+64); the containing cell is the
    deepest cell whose particle range holds every member (brute force over all cells)."""
    from oracle import hilbert
    from paper_1112_4539_amd import inputs
    pos, mass = inputs.clumpy(3000, 9)
    T = oracle.Tree(pos, mass)
    order = hilbert.walk_positions(pos, mass)
    X = learn.features(T, pos, mass, order)
    n = len(pos)
    rho_mean = T.M[0] / T.L ** 3
    for g in range((n + 63) // 64):
        mem = order[64 * g: 64 * g + 64]
        holds = [c for c in range(len(T.M)) if np.all((T.first[c] <= mem) & (mem < T.first[c] + T.count[c]))]
        c = max(holds, key=lambda k: (T.level[k], k))
        ps = pos[T.perm[mem]]
        h = max(np.max(ps.max(0) - ps.min(0)) / 2, T.L * 2.0 ** -22)
        np.testing.assert_allclose(X[g, 5], np.log10(T.M[c] / T.l[c] ** 3 / rho_mean), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(X[g, 7], np.log2(T.l[c] / h), rtol=1e-12)
        w = mass[T.perm[mem]]
        com = (w[:, None] * ps).sum(0) / w.sum()
        np.testing.assert_allclose(X[g, 4], np.linalg.norm(com - 0.5 * (ps.max(0) + ps.min(0))) / h, rtol=1e-9,
                                   atol=1e-12)
    # the Morton order as the walk order gives the Morton groups
    np.testing.assert_array_equal(learn.features(T, pos, mass, np.arange(n)), learn.features(T, pos, mass))


def test_group_rms_walk_groups():
    # per-particle relative errors e_i planted exactly; group g = order[64g, 64g+64)
    n = 300
    rng = np.random.default_rng(10)
    ref = rng.normal(size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    e = rng.uniform(1e-4, 1e-2, n)
    acc = ref + (e * np.linalg.norm(ref, axis=1))[:, None] * d
    perm = rng.permutation(n)
    order = rng.permutation(n)
    r = learn.group_rms(acc, ref, perm, order)
    for g in range((n + 63) // 64):
        mem = perm[order[64 * g: 64 * g + 64]]
        np.testing.assert_allclose(r[g], np.sqrt(np.mean(e[mem] ** 2)), rtol=1e-9)
