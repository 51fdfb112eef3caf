"""GPU parity of the batched forest, the persistent walk, graph replays and the autotuner.

A forest of K clusters must give every cluster exactly what the same cluster
built alone gives (bit for bit: node records, forces, list counts and hashes),
and every cluster's lists and forces must match the CPU oracle run on that
cluster alone.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1112_4539_amd import inputs
from tests.util import check_forces, pot_err

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
F64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bh():
    import paper_1112_4539_amd as bh
    bh.load()
    assert torch.cuda.is_available()
    return bh


def _dt(prec):
    return torch.float32 if prec == "fp32" else torch.float64


def _small_forest():
    """Clusters of awkward sizes: empty, one particle, coincident, ragged, a wave edge."""
    rng = np.random.default_rng(77)
    parts = [
        np.zeros((0, 3)),
        np.array([[0.5, -1.0, 2.0]]),
        np.full((70, 3), 0.125),                      # one bucket leaf
        inputs.plummer(300, None, rng=rng)[0],
        np.zeros((0, 3)),
        inputs.plummer(1000, None, rng=rng)[0] * 3.0 + 5.0,
        rng.random((64, 3)),
        rng.random((2, 3)),
        inputs.plummer(129, None, rng=rng)[0],
    ]
    sizes = np.array([len(p) for p in parts], np.int64)
    pos = np.concatenate(parts)
    mass = rng.random(len(pos)) + 0.5
    off = np.zeros(len(parts) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    return pos, mass, off


def _forest_vs_alone(bh, pos, mass, off, prec, theta, eps, clusters=None, check_nodes=True, tpl=1):
    dt = _dt(prec)
    gp = torch.tensor(pos, dtype=dt, device="cuda")
    gm = torch.tensor(mass, dtype=dt, device="cuda")
    go = torch.tensor(off, dtype=torch.int64, device="cuda")
    F = bh.build_forest(gp, gm, go)
    F.set_walk_config(targets_per_lane=tpl)
    F.check()
    st = F.walk_stats(theta, eps)
    a_f, p_f = F.forces(theta, eps)
    torch.cuda.synchronize()
    assert torch.equal(a_f, st["acc"]) and torch.equal(p_f, st["pot"])
    roots = F.roots().cpu().numpy()
    rec = F.export()[0] if check_nodes else None
    K = len(off) - 1
    for k in (range(K) if clusters is None else clusters):
        b, e = int(off[k]), int(off[k + 1])
        if e == b:
            assert roots[k] == roots[k + 1]
            continue
        T = bh.Tree(gp[b:e].contiguous(), gm[b:e].contiguous())
        s1 = T.walk_stats(theta, eps)
        assert torch.equal(s1["acc"], st["acc"][b:e]), k
        assert torch.equal(s1["pot"], st["pot"][b:e]), k
        assert torch.equal(s1["counts"], st["counts"][b:e]), k
        assert torch.equal(s1["hash"], st["hash"][b:e]), k
        if check_nodes:
            r1, perm1 = T.export()
            sub = rec[roots[k]:roots[k + 1]]
            assert len(sub) == len(r1), k
            for f in ("com", "M", "l", "s", "count", "meta"):
                np.testing.assert_array_equal(sub[f], r1[f])
            np.testing.assert_array_equal(sub["next"] - roots[k], r1["next"])
            np.testing.assert_array_equal(sub["first"] - b, r1["first"])
    return F, st


@pytest.mark.parametrize("prec,tpl", [("fp32", 1), ("fp64", 1), ("fp32", 2)])
def test_forest_equals_clusters_alone(bh, prec, tpl):
    say(f"[forest] small awkward clusters {prec}, {tpl} targets per lane in the forest")
    pos, mass, off = _small_forest()
    _forest_vs_alone(bh, pos, mass, off, prec, 0.6, 0.01, tpl=tpl)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_forest_against_oracle(bh, prec):
    say(f"[forest] oracle per cluster {prec}")
    pos, mass, off = _small_forest()
    dt = _dt(prec)
    npdt = np.float32 if prec == "fp32" else np.float64
    F = bh.build_forest(torch.tensor(pos, dtype=dt, device="cuda"), torch.tensor(mass, dtype=dt, device="cuda"),
                        torch.tensor(off, device="cuda"))
    st = F.walk_stats(0.6, 0.01, maxlen=1100)
    tol = F32_TOL if prec == "fp32" else F64_TOL
    for k in range(len(off) - 1):
        b, e = int(off[k]), int(off[k + 1])
        if e == b:
            continue
        p64 = pos[b:e].astype(npdt).astype(np.float64)
        m64 = mass[b:e].astype(npdt).astype(np.float64)
        w = oracle.Tree(p64, m64).walk(0.6, 0.01, maxlen=1100)
        cnt = st["counts"][b:e].cpu().numpy()
        np.testing.assert_array_equal(cnt[:, 0], w["n_pp"])
        np.testing.assert_array_equal(cnt[:, 1], w["n_pc"])
        np.testing.assert_array_equal(st["hash"][b:e].cpu().numpy().view(np.uint64), w["hash"])
        np.testing.assert_array_equal(st["lists"][b:e].cpu().numpy(), w["lists"])
        acc = st["acc"][b:e].cpu().numpy().astype(np.float64)
        pot = st["pot"][b:e].cpu().numpy().astype(np.float64)
        check_forces(acc, w["acc"], w["amag"], tol, f"cluster {k}", log=say)
        assert pot_err(pot, w["pot"]).max() <= tol, k


@pytest.mark.parametrize("K,smax", [(300, 48), (2047, 48), (2048, 48), (3001, 48), (140_000, 4)])
def test_forest_many_clusters(bh, K, smax):
    """Cluster counts around the sort's two ways of finding an item's cluster:
    a search over the offsets staged in LDS (K + 1 <= 2048) and the per-index
    cluster array above that; both need two cluster digits.  Beyond 131,072
    clusters the Hilbert target order's key needs an odd number of passes."""
    say(f"[forest] {K} small clusters fp32")
    rng = np.random.default_rng(K)
    sizes = rng.integers(0, smax, K)
    sizes[rng.choice(K, K // 10, replace=False)] = 0
    sizes[-1] = 5
    off = np.zeros(K + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    ctr = rng.normal(size=(K, 3)) * 10.0
    pos = rng.normal(size=(n, 3)) * 0.1 + np.repeat(ctr, sizes, axis=0)
    mass = rng.random(n) + 0.5
    picks = sorted(set(rng.choice(K, 12, replace=False).tolist()) | {0, 255, 256, K - 1})
    F, st = _forest_vs_alone(bh, pos, mass, off, "fp32", 0.6, 0.01, clusters=picks)
    roots = F.roots().cpu().numpy()
    # every cluster's subtree holds exactly its own particles
    rec = F.export()[0]
    for k in range(K):
        if sizes[k]:
            assert rec[roots[k]]["count"] == sizes[k] and rec[roots[k]]["first"] == off[k], k
        else:
            assert roots[k] == roots[k + 1], k


def test_forest_bad_offsets_reported(bh):
    say("[forest] invalid offsets")
    pos = torch.rand((100, 3), device="cuda")
    mass = torch.ones(100, device="cuda")
    for off in ([0, 60, 50, 100], [0, 50, 101], [1, 50, 100], [0, 50, 99]):
        F = bh.build_forest(pos, mass, torch.tensor(off, device="cuda"))
        with pytest.raises(ValueError):
            F.check()
        F.forces(0.5, 0.01)       # runs to completion; the results are not meaningful
        torch.cuda.synchronize()


def test_forest_full_size(bh):
    """512 log-uniform Plummer clusters (seed 3, ~8M particles), theta 0.5, eps 0.01, FP32."""
    say("[forest] 512 clusters full size")
    pos, mass, off = inputs.clusters(512, 3)
    K = len(off) - 1
    sizes = np.diff(off)
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0, K - 1, 257})
    F, st = _forest_vs_alone(bh, pos, mass, off, "fp32", 0.5, 0.01, clusters=picks, check_nodes=False)
    # oracle on sampled targets of two clusters
    for k in (picks[0], picks[-1]):
        b, e = int(off[k]), int(off[k + 1])
        p64 = pos[b:e].astype(np.float32).astype(np.float64)
        m64 = mass[b:e].astype(np.float32).astype(np.float64)
        tg = inputs.sample_targets(e - b, min(512, e - b), 300 + k)
        w = oracle.Tree(p64, m64).walk(0.5, 0.01, targets=tg)
        cnt = st["counts"][b:e].cpu().numpy()[tg]
        np.testing.assert_array_equal(cnt[:, 0], w["n_pp"])
        np.testing.assert_array_equal(cnt[:, 1], w["n_pc"])
        np.testing.assert_array_equal(st["hash"][b:e].cpu().numpy().view(np.uint64)[tg], w["hash"])
        acc = st["acc"][b:e].cpu().numpy()[tg].astype(np.float64)
        check_forces(acc, w["acc"], w["amag"], F32_TOL, "forest", log=say)
    # persistent walk of the whole forest: same bits
    a0, p0 = st["acc"], st["pot"]
    for tpl in (1, 2):
        F.set_walk_config(4, 0, 0, 16, 1, tpl)
        a1, p1 = F.forces(0.5, 0.01)
        assert torch.equal(a1, a0) and torch.equal(p1, p0)


@pytest.mark.parametrize("forest,order", [(False, 0), (True, 0), (False, 2), (True, 2)])
def test_graph_replays_match_eager(bh, forest, order):
    say(f"[graph] replays forest={forest} target order {order}")
    if forest:
        pos, mass, off = inputs.clusters(24, 11, nmin=64, nmax=4096)
    else:
        pos, mass = inputs.plummer(20_000, 5)
        off = None
    gp = torch.tensor(pos, dtype=torch.float32, device="cuda")
    gm = torch.tensor(mass, dtype=torch.float32, device="cuda")
    go = None if off is None else torch.tensor(off, device="cuda")
    T = bh.Tree(gp, gm, offsets=go)
    T.set_walk_config(2, 0, order, 16, 1, 2)
    acc = torch.zeros((len(pos), 3), dtype=torch.float32, device="cuda")
    pot = torch.zeros((len(pos),), dtype=torch.float32, device="cuda")
    G = T.graph(0.5, 0.01, acc, pot)
    # an eager walk between the capture and the first replay
    a0, p0 = T.forces(0.5, 0.01)
    E0 = bh.Tree(gp.clone(), gm.clone(), offsets=go)
    a0e, p0e = E0.forces(0.5, 0.01)
    torch.cuda.synchronize()
    assert torch.equal(a0, a0e) and torch.equal(p0, p0e)
    rng = np.random.default_rng(5)
    for rep in range(4):
        # new contents in the same input tensors, then one replay
        scale = float(rng.uniform(0.5, 2.0))
        gp.copy_(torch.tensor(pos * scale, dtype=torch.float32, device="cuda"))
        acc.fill_(float("nan"))
        G.launch()
        torch.cuda.synchronize()
        E = bh.Tree(gp.clone(), gm.clone(), offsets=go)
        a_e, p_e = E.forces(0.5, 0.01)
        torch.cuda.synchronize()
        assert torch.equal(acc, a_e) and torch.equal(pot, p_e), rep


def test_autotune_keeps_results(bh):
    say("[autotune] clumpy 200k fp32")
    pos, mass = inputs.clumpy(200_000, 13)
    T = bh.Tree(torch.tensor(pos, dtype=torch.float32, device="cuda"),
                torch.tensor(mass, dtype=torch.float32, device="cuda"))
    ref = T.forces(0.5, 1e-4)
    a_ref, p_ref = ref[0].clone(), ref[1].clone()
    best, tried = T.autotune(0.5, 1e-4, reps=1)
    say(f"  best {best}  ({len(tried)} tried)")
    assert len(tried) >= 8   # 1 + 1 + 1 + 2 + 3, plus 2 more when the block-order walk wins
    assert best["ms"] == min(t["ms"] for t in tried)
    a, p = T.forces(0.5, 1e-4)
    assert torch.equal(a, a_ref) and torch.equal(p, p_ref)
