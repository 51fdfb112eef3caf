"""GPU parity: the HIP library against the CPU FP64 oracle, element by element.

Tree: node set, preorder numbering, next pointers and FP64 moments bit-exact.
Walk: interaction lists identical (full dumps at small n, per-particle count +
ordered-list hash at full size), forces within 1e-12 (FP64) / 1e-5 (FP32)
relative per particle, with the cancellation floor of ``util.force_err``.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1112_4539_amd import inputs
from tests.util import walk_slots, check_forces, force_err, pot_err, tree_cases, widen

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


def _np_dtype(prec):
    return np.float32 if prec == "fp32" else np.float64


def _gpu(pos, mass, prec):
    dt = torch.float32 if prec == "fp32" else torch.float64
    return (torch.tensor(pos, dtype=dt, device="cuda"), torch.tensor(mass, dtype=dt, device="cuda"))


def _seen(pos, mass, prec):
    """The values the GPU sees, widened exactly to float64 for the oracle."""
    t = _np_dtype(prec)
    return pos.astype(t).astype(np.float64), mass.astype(t).astype(np.float64)


def _compare_trees(bh, pos, mass, prec):
    gp, gm = _gpu(pos, mass, prec)
    T = bh.Tree(gp, gm)
    rec, perm = T.export()
    p64, m64 = _seen(pos, mass, prec)
    O = oracle.Tree(p64, m64)
    assert len(rec) == O.n_nodes
    np.testing.assert_array_equal(perm, O.perm)
    np.testing.assert_array_equal(rec["meta"] & 1, O.leaf)
    np.testing.assert_array_equal(rec["meta"] >> 8, O.level)
    np.testing.assert_array_equal(rec["first"], O.first)
    np.testing.assert_array_equal(rec["count"], O.count)
    np.testing.assert_array_equal(rec["next"], O.next)
    np.testing.assert_array_equal(rec["com"], O.com)
    np.testing.assert_array_equal(rec["M"], O.M)
    np.testing.assert_array_equal(rec["l"], O.l)
    np.testing.assert_array_equal(rec["s"], O.s)
    return T, O


@pytest.mark.parametrize("name", sorted(tree_cases()))
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tree_bitexact_small(bh, name, prec):
    say(f"[tree] case={name} prec={prec}")
    pos = tree_cases()[name]
    mass = np.random.default_rng(len(pos)).random(len(pos)) + 0.5
    _compare_trees(bh, pos, mass, prec)


@pytest.mark.parametrize("which,prec", [("plummer4k", "fp64"), ("plummer4k", "fp32"), ("clumpy", "fp32")])
def test_tree_bitexact_workloads(bh, which, prec):
    say(f"[tree] workload={which} prec={prec}")
    if which == "plummer4k":
        pos, mass = inputs.plummer(4096, 0)
    else:
        pos, mass = inputs.clumpy(200_003, 21)      # ragged: not a multiple of any tile
    _compare_trees(bh, pos, mass, prec)


def _walk_compare(bh, pos, mass, prec, theta, eps, targets=None, maxlen=0, theta_group=None, tpl=1,
                  target_order=2):
    gp, gm = _gpu(pos, mass, prec)
    T = bh.Tree(gp, gm)
    T.set_walk_config(targets_per_lane=tpl, target_order=target_order)
    tg_t = None if theta_group is None else torch.tensor(theta_group, dtype=torch.float32, device="cuda")
    out = T.walk_stats(theta, eps, theta_group=tg_t, maxlen=maxlen)
    acc_f, pot_f = T.forces(theta, eps, theta_group=tg_t)
    torch.cuda.synchronize()
    # the plain force walk gives the very same numbers as the instrumented one
    assert torch.equal(acc_f, out["acc"]) and torch.equal(pot_f, out["pot"])
    p64, m64 = _seen(pos, mass, prec)
    O = oracle.Tree(p64, m64)
    idx = np.arange(len(pos)) if targets is None else targets
    tpt = None
    if theta_group is not None:
        # theta of the target's walk group (runs of 64 of the Hilbert order, or of the Morton order)
        if target_order == 2:
            slots = walk_slots(p64, m64)
        else:
            slots = np.empty(len(pos), np.int64)
            slots[O.perm] = np.arange(len(pos))
        tpt = np.asarray(theta_group, np.float32).astype(np.float64)[slots[idx] // 64]
    w = O.walk(theta, eps, targets=idx, theta_per_target=tpt, maxlen=maxlen)
    cnt = out["counts"].cpu().numpy()[idx]
    np.testing.assert_array_equal(cnt[:, 0], w["n_pp"])
    np.testing.assert_array_equal(cnt[:, 1], w["n_pc"])
    np.testing.assert_array_equal(out["hash"].cpu().numpy().view(np.uint64)[idx], w["hash"])
    if maxlen:
        np.testing.assert_array_equal(out["lists"].cpu().numpy()[idx], w["lists"])
    acc = out["acc"].cpu().numpy()[idx]
    pot = out["pot"].cpu().numpy()[idx]
    return acc, pot, w


@pytest.mark.parametrize("tpl", [1, 2])
def test_lists_and_forces_plummer4k_fp64(bh, tpl):
    say(f"[walk] plummer4k fp64 theta=0.5 full list dump, {tpl} targets per lane")
    pos, mass = inputs.plummer(4096, 0)
    acc, pot, w = _walk_compare(bh, pos, mass, "fp64", 0.5, 0.01, maxlen=4096, tpl=tpl)
    check_forces(acc, w["acc"], w["amag"], F64_TOL, "fp64", log=say)
    say(f"  bit-exact share {np.mean(np.all(acc == w['acc'], axis=1)):.4f}")
    assert pot_err(pot, w["pot"]).max() <= F64_TOL


@pytest.mark.parametrize("tpl", [1, 2])
@pytest.mark.parametrize("theta", [0.3, 0.5, 0.75])
def test_lists_and_forces_plummer4k_fp32(bh, theta, tpl):
    say(f"[walk] plummer4k fp32 theta={theta} full list dump, {tpl} targets per lane")
    pos, mass = inputs.plummer(4096, 0)
    acc, pot, w = _walk_compare(bh, pos, mass, "fp32", theta, 0.01, maxlen=4096, tpl=tpl)
    check_forces(acc, w["acc"], w["amag"], F32_TOL, "fp32", log=say)
    assert pot_err(pot, w["pot"]).max() <= F32_TOL


@pytest.mark.parametrize("prec,tpl", [("fp64", 1), ("fp32", 1), ("fp32", 2)])
def test_unsoftened(bh, prec, tpl):
    """eps = 0, the unsoftened pair term of Eq. (1) (the walk's variant without softening): full
    list dumps and forces against the oracle, with a leaf of five coincident particles, which add
    nothing to each other (a pair at r = 0 has no defined force without softening)."""
    say(f"[walk] plummer4k {prec} eps=0 full list dump, {tpl} targets per lane")
    pos, mass = inputs.plummer(4096, 0)
    pos = pos.copy()
    pos[100:104] = pos[99]
    acc, pot, w = _walk_compare(bh, pos, mass, prec, 0.5, 0.0, maxlen=4096, tpl=tpl)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    tol = F32_TOL if prec == "fp32" else F64_TOL
    check_forces(acc, w["acc"], w["amag"], tol, f"eps=0 {prec}", log=say)
    assert pot_err(pot, w["pot"]).max() <= tol


@pytest.mark.parametrize("prec,theta", [("fp64", 1.1), ("fp32", 1.1), ("fp32", 1.15)])
def test_lists_theta_above_one(bh, prec, theta):
    """theta in (1, 2/sqrt(3)): a cell holding the target can pass the opening
    test, and the walk must exclude it by its particle range (the guarded path)."""
    say(f"[walk] plummer4k {prec} theta={theta} full list dump (guarded walk)")
    pos, mass = inputs.plummer(4096, 0)
    acc, pot, w = _walk_compare(bh, pos, mass, prec, theta, 0.01, maxlen=4096)
    tol = F32_TOL if prec == "fp32" else F64_TOL
    check_forces(acc, w["acc"], w["amag"], tol, prec, log=say)
    assert pot_err(pot, w["pot"]).max() <= tol


@pytest.mark.parametrize("prec,tpl,order", [("fp32", 1, 2), ("fp32", 2, 2), ("fp64", 1, 2), ("fp32", 1, 0),
                                            ("fp64", 1, 0)])
def test_theta_per_group(bh, prec, tpl, order):
    """Per-group theta in [0.2, 1.15], one value per walk group (runs of 64 of the Hilbert order,
    or of the Morton order): the FP32 walk reads its own node copy (l, s), the FP64 walk the plain
    nodes; lists must equal the oracle's per-target-theta walk in both."""
    say(f"[walk] per-group theta, clumpy 50k {prec}, {tpl} targets per lane, target order {order}")
    pos, mass = inputs.clumpy(50_000, 31)
    g = (len(pos) + 63) // 64
    tg = np.random.default_rng(3).uniform(0.2, 1.15, g).astype(np.float32)
    acc, pot, w = _walk_compare(bh, pos, mass, prec, 0.5, 1e-4, theta_group=tg, tpl=tpl, target_order=order)
    tol = F32_TOL if prec == "fp32" else F64_TOL
    check_forces(acc, w["acc"], w["amag"], tol, prec, log=say)
    assert pot_err(pot, w["pot"]).max() <= tol


def test_direct_fp64_matches_definition(bh):
    say("[direct] plummer4k fp64")
    pos, mass = inputs.plummer(4096, 0)
    gp, gm = _gpu(pos, mass, "fp64")
    tg = torch.arange(4096, device="cuda")
    acc, pot = bh.direct(gp, gm, 0.01, tg)
    a_ref, p_ref, amag = oracle.direct(pos, mass, 0.01)
    acc = acc.cpu().numpy()
    check_forces(acc, a_ref, amag, F64_TOL, "direct fp64", log=say)
    say(f"  bit-exact share {np.mean(acc == a_ref):.4f}")
    assert pot_err(pot.cpu().numpy(), p_ref).max() <= F64_TOL


def test_direct_fp32_close_to_fp64(bh):
    say("[direct] plummer 20k fp32 vs fp64")
    pos, mass = inputs.plummer(20_000, 5)
    tg = torch.tensor(inputs.sample_targets(20_000, 2000, 5), device="cuda")
    a32, _ = bh.direct(*_gpu(pos, mass, "fp32"), 0.01, tg)
    p64, m64 = _seen(pos, mass, "fp32")
    a64, _, amag = oracle.direct(p64, m64, 0.01, targets=tg.cpu().numpy())
    assert np.quantile(force_err(a32.cpu().numpy(), a64, amag), 0.99) < 1e-5


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_permutation_and_scaling_bitexact(bh, prec):
    say(f"[invariance] plummer 30k {prec}")
    pos, mass = inputs.plummer(30_000, 8)
    perm = np.random.default_rng(4).permutation(len(pos))
    T1 = bh.Tree(*_gpu(pos, mass, prec))
    a1, p1 = T1.forces(0.6, 0.01)
    T2 = bh.Tree(*_gpu(pos[perm], mass[perm], prec))
    a2, p2 = T2.forces(0.6, 0.01)
    pt = torch.tensor(perm, device="cuda")
    assert torch.equal(a2, a1[pt]) and torch.equal(p2, p1[pt])
    T3 = bh.Tree(*_gpu(pos * 2.0, mass * 8.0, prec))
    a3, p3 = T3.forces(0.6, 0.02)
    assert torch.equal(a3, 2 * a1) and torch.equal(p3, 4 * p1)


def test_launch_shapes_and_target_order_bitexact(bh):
    say("[invariance] launch shapes, clumpy 100k fp32")
    pos, mass = inputs.clumpy(100_000, 9)
    T = bh.Tree(*_gpu(pos, mass, "fp32"))
    ref = T.forces(0.5, 1e-4)
    for wpb in (1, 2, 4):
        for chunk in (0, 4, 16):
            for order in (0, 1, 2):
                for share in (0, 24, 64):
                    for pers in (0, 1):
                        for tpl in (1, 2):
                            if pers and chunk:
                                continue  # the block remap does not apply to the persistent walk
                            T.set_walk_config(wpb, chunk, order, share, pers, tpl)
                            a, p = T.forces(0.5, 1e-4)
                            assert torch.equal(a, ref[0]) and torch.equal(p, ref[1]), (wpb, chunk, order, share,
                                                                                       pers, tpl)


def test_walk_config_values(bh):
    """The launch-shape knobs reject values outside their ranges; -1 (automatic
    XCD runs) and every target order give the same bits."""
    say("[config] knob ranges, plummer 20k fp32 and fp64")
    pos, mass = inputs.plummer(20_000, 21)
    for prec in ("fp32", "fp64"):
        T = bh.Tree(*_gpu(pos, mass, prec))
        ref = T.forces(0.5, 0.01)
        for bad in (dict(xcd_chunk=-2), dict(target_order=3), dict(target_order=-1), dict(waves_per_block=3),
                    dict(lds_share=65), dict(persistent=2), dict(targets_per_lane=3)):
            with pytest.raises(ValueError):
                T.set_walk_config(**bad)
        for chunk in (-1, 0, 1, 1024, 1 << 20):
            for order in (0, 1, 2):
                T.set_walk_config(xcd_chunk=chunk, target_order=order)
                a, p = T.forces(0.5, 0.01)
                assert torch.equal(a, ref[0]) and torch.equal(p, ref[1]), (prec, chunk, order)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_edge_cases(bh, prec):
    say(f"[edge] {prec}")
    dt = torch.float32 if prec == "fp32" else torch.float64
    # empty
    T = bh.Tree(torch.empty((0, 3), dtype=dt, device="cuda"), torch.empty((0,), dtype=dt, device="cuda"))
    a, p = T.forces(0.5, 0.01)
    assert a.shape == (0, 3) and T.stats()["n_nodes"] == 0
    # one particle: no force
    T = bh.Tree(torch.tensor([[0.3, 0.1, -2.0]], dtype=dt, device="cuda"), torch.tensor([2.0], dtype=dt, device="cuda"))
    a, p = T.forces(0.5, 0.01)
    assert torch.all(a == 0) and torch.all(p == 0)
    # two particles: the closed form (dx = (1,2,2), eps = 4 -> r = 5)
    T = bh.Tree(torch.tensor([[0, 0, 0], [1, 2, 2]], dtype=dt, device="cuda"),
                torch.tensor([1.0, 0.75], dtype=dt, device="cuda"))
    a, p = T.forces(0.5, 4.0)
    np.testing.assert_allclose(a.cpu().numpy()[0], 0.75 * np.array([1, 2, 2]) / 125, rtol=4e-7)
    np.testing.assert_allclose(p.cpu().numpy(), [-0.15, -0.2], rtol=4e-7)
    # all coincident: one bucket leaf, potentials -m/eps, zero accelerations
    pos = torch.full((70, 3), 0.25, dtype=dt, device="cuda")
    mass = torch.full((70,), 0.5, dtype=dt, device="cuda")
    T = bh.Tree(pos, mass)
    a, p = T.forces(0.5, 0.5)
    assert T.stats()["n_nodes"] == 1
    assert torch.all(a == 0)
    np.testing.assert_allclose(p.cpu().numpy(), -69 * 0.5 / 0.5, rtol=1e-6)
    # invalid parameters are rejected on the host
    for bad in (0.0, -0.1, 1.2, float("nan")):
        with pytest.raises(ValueError):
            T.forces(bad, 0.01)
    with pytest.raises(ValueError):
        T.forces(0.5, -1.0)
    # non-finite inputs are reported by the check pass
    pos = torch.rand((100, 3), dtype=dt, device="cuda")
    pos[17, 1] = float("nan")
    T = bh.Tree(pos, torch.ones(100, dtype=dt, device="cuda"))
    with pytest.raises(ValueError):
        T.check()


@pytest.mark.parametrize("name,theta,tpl", [("plummer1m", 0.3, 1), ("plummer1m", 0.5, 1), ("plummer1m", 0.75, 1),
                                            ("clumpy4m", 0.5, 1), ("clumpy4m", 0.35, 2)])
def test_full_size_sampled(bh, name, theta, tpl):
    say(f"[full] {name} theta={theta} (sampled targets), {tpl} targets per lane")
    pos, mass, spec = inputs.make(name)
    tg = inputs.sample_targets(len(pos), 2048, spec["seed"] + 100)
    acc, pot, w = _walk_compare(bh, pos, mass, "fp32", theta, spec["eps"], targets=tg, tpl=tpl)
    check_forces(acc, w["acc"], w["amag"], F32_TOL, name, log=say)
    say(f"  mean L {np.mean(w['n_pp'] + w['n_pc']):.0f}")
    assert pot_err(pot, w["pot"]).max() <= F32_TOL


def test_walk_copy_above_4gib(bh):
    """n = 2^25 + 4097 particles: the walk copy (2n + 1 records of 64 bytes) passes 4 GiB, so the walk
    reads its records with 64-bit addresses instead of 32-bit offsets; sampled targets against the oracle."""
    n = (1 << 25) + 4097
    say(f"[full] uniform cube n={n} theta=0.6 (sampled targets): 64-bit record addressing")
    rng = np.random.default_rng(7)
    pos = rng.random((n, 3))
    mass = np.full(n, 1.0 / n)
    tg = inputs.sample_targets(n, 256, 17)
    acc, pot, w = _walk_compare(bh, pos, mass, "fp32", 0.6, 1e-3, targets=tg)
    check_forces(acc, w["acc"], w["amag"], F32_TOL, "cube 2^25+4097", log=say)
    say(f"  mean L {np.mean(w['n_pp'] + w['n_pc']):.0f}")
    assert pot_err(pot, w["pot"]).max() <= F32_TOL


def test_theta_per_group_invalid_values(bh):
    """Per-group theta values that are not finite or outside (0, 2/sqrt(3)) are replaced by 0.5 on the
    device and reported by the check; the other groups are untouched, and a walk with valid values
    clears the report."""
    say("[walk] per-group theta with invalid entries, clumpy 20k fp32")
    pos, mass = inputs.clumpy(20_000, 33)
    g = (len(pos) + 63) // 64
    tg = np.random.default_rng(4).uniform(0.3, 1.0, g).astype(np.float32)
    bad = {3: np.nan, 7: 0.0, 11: -0.5, 13: 1.2, 17: np.inf, 19: -np.inf}
    for k, v in bad.items():
        tg[k] = v
    gp, gm = _gpu(pos, mass, "fp32")
    T = bh.Tree(gp, gm)
    out = T.walk_stats(0.5, 1e-4, theta_group=torch.tensor(tg, device="cuda"))
    with pytest.raises(ValueError, match="theta"):
        T.check()
    fixed = tg.copy()
    for k in bad:
        fixed[k] = 0.5
    p64, m64 = _seen(pos, mass, "fp32")
    O = oracle.Tree(p64, m64)
    w = O.walk(0.5, 1e-4, theta_per_target=fixed.astype(np.float64)[walk_slots(p64, m64) // 64])
    np.testing.assert_array_equal(out["hash"].cpu().numpy().view(np.uint64), w["hash"])
    check_forces(out["acc"].cpu().numpy(), w["acc"], w["amag"], F32_TOL, "fallback", log=say)
    T.forces(0.5, 1e-4, theta_group=torch.tensor(fixed, device="cuda"))
    T.check()


def test_theta_per_group_full_size(bh):
    """The per-group theta walk at the size the learned-theta runs use it (clumpy 4M, FP32), theta_g drawn
    in [0.2, 1.15]: counts, ordered-list hashes and forces of 2048 sampled targets against the oracle's
    per-target-theta walk."""
    say("[full] clumpy4m per-group theta in [0.2, 1.15] fp32 (sampled targets)")
    pos, mass, spec = inputs.make("clumpy4m")
    g = (len(pos) + 63) // 64
    thg = np.random.default_rng(41).uniform(0.2, 1.15, g).astype(np.float32)
    tg = inputs.sample_targets(len(pos), 2048, spec["seed"] + 200)
    acc, pot, w = _walk_compare(bh, pos, mass, "fp32", 0.5, spec["eps"], targets=tg, theta_group=thg)
    check_forces(acc, w["acc"], w["amag"], F32_TOL, "clumpy4m per-group", log=say)
    assert pot_err(pot, w["pot"]).max() <= F32_TOL


def test_fp64_walk_full_size(bh):
    """The FP64 walk (the accuracy reference of the Plummer sweep) at N = 1,048,576, theta = 0.5:
    counts, hashes and forces of 2048 sampled targets against the oracle at 1e-12."""
    say("[full] plummer1m fp64 theta=0.5 (sampled targets)")
    pos, mass, spec = inputs.make("plummer1m")
    tg = inputs.sample_targets(len(pos), 2048, spec["seed"] + 300)
    acc, pot, w = _walk_compare(bh, pos, mass, "fp64", 0.5, spec["eps"], targets=tg)
    check_forces(acc, w["acc"], w["amag"], F64_TOL, "plummer1m fp64", log=say)
    assert pot_err(pot, w["pot"]).max() <= F64_TOL


@pytest.mark.parametrize("b,prec", [(1, "fp32"), (2, "fp32"), (3, "fp64"), (4, "fp32"), (5, "fp64")])
def test_hilbert_walk_order_on_a_lattice(bh, b, prec):
    """One particle in each cell of the 2^b grid of the root cube: the Hilbert target order visits
    every particle once, and consecutive targets sit in face-adjacent cells (the defining property
    of a Hilbert curve, which no Morton or row-major order has).  The Morton order is checked to
    fail it."""
    say(f"[hilbert] lattice 2^{b} per axis, {prec}")
    k = 1 << b
    g = (np.arange(k) + 0.5) / k
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(b)
    perm = rng.permutation(len(pos))
    pos = pos[perm]
    mass = np.full(len(pos), 1.0 / len(pos))
    T = bh.Tree(*_gpu(pos, mass, prec))
    idx = (np.floor(pos * k)).astype(np.int64)
    for order, adjacent in ((2, True), (0, False)):
        T.set_walk_config(target_order=order)
        w = T.walk_order().cpu().numpy().astype(np.int64)
        assert np.array_equal(np.sort(w), np.arange(len(pos)))
        steps = np.abs(np.diff(idx[w], axis=0)).sum(1)
        if adjacent:
            assert np.all(steps == 1), (order, np.unique(steps))
        else:
            assert steps.max() > 1


@pytest.mark.parametrize("case,prec", [("clumpy", "fp32"), ("duplicates", "fp32"), ("plummer", "fp64"),
                                       ("forest", "fp32")])
def test_hilbert_walk_order_matches_oracle(bh, case, prec):
    """The Hilbert target order (Sec. 5's Peano-Hilbert remark) element by element against the
    oracle's (oracle/hilbert.py: Skilling's transform of the cell ten levels below the root cube,
    ties in Morton order; per cluster with fewer levels in a forest)."""
    from oracle import hilbert
    say(f"[hilbert] walk order vs oracle: {case} {prec}")
    offsets = None
    if case == "clumpy":
        pos, mass = inputs.clumpy(150_001, 12)
    elif case == "duplicates":
        pos, mass = inputs.clumpy(60_000, 13)
        pos[40_000:] = pos[:20_000]          # coincident pairs: ties of the key
    elif case == "plummer":
        pos, mass = inputs.plummer(70_000, 14)
    else:
        rng = np.random.default_rng(15)
        sizes = rng.integers(1, 3000, 40)
        sizes[3] = 1
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pos = rng.random((offsets[-1], 3)) + np.repeat(rng.random((40, 3)) * 10, sizes, axis=0)
        mass = rng.uniform(0.5, 1.5, offsets[-1])
    gp, gm = _gpu(pos, mass, prec)
    if offsets is None:
        T = bh.Tree(gp, gm)
    else:
        T = bh.build_forest(gp, gm, torch.tensor(offsets, device="cuda"))
    T.set_walk_config(target_order=2)
    got = T.walk_order().cpu().numpy().astype(np.int64)
    # the oracle sees exactly the values the GPU tree is built from
    p64 = gp.double().cpu().numpy()
    want = hilbert.walk_order(p64, gm.double().cpu().numpy(), offsets)
    bad = np.flatnonzero(got != want)
    say(f"  n={len(pos)} mismatches={len(bad)}")
    assert len(bad) == 0, bad[:10]
