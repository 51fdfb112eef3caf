"""Walks with theta per walk group from a table of levels (bh_forces_theta_levels, bh_theta_quantize).

Theta is the opening parameter of Eq. (2); a level walk gives walk group g (the 64 targets at
[64g, 64g+64) of the walk order) theta = level_theta[group_level[g]].  Its lists must equal the
oracle's per-target-theta walk, and its results those of bh_forces_theta with the same values.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1112_4539_amd import inputs
from tests.util import check_forces, pot_err, walk_slots

pytestmark = pytest.mark.gpu
F32_TOL, F64_TOL = 1e-5, 1e-12
LEVELS = [0.25, 0.4, 0.55, 0.7, 0.9, 1.05]   # one above 1: cells holding their target are excluded by range


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bh():
    import paper_1112_4539_amd as bh
    bh.load()
    assert torch.cuda.is_available()
    return bh


def _tree(bh, pos, mass, prec="fp32", order=2, offsets=None):
    dt = torch.float32 if prec == "fp32" else torch.float64
    gp = torch.tensor(pos, dtype=dt, device="cuda")
    gm = torch.tensor(mass, dtype=dt, device="cuda")
    T = bh.Tree(gp, gm) if offsets is None else bh.build_forest(gp, gm, torch.tensor(offsets, device="cuda"))
    T.set_walk_config(target_order=order)
    return T, gp.double().cpu().numpy(), gm.double().cpu().numpy()


def _levels(n, seed, n_levels=len(LEVELS)):
    g = (n + 63) // 64
    return torch.tensor(np.random.default_rng(seed).integers(0, n_levels, g).astype(np.uint8), device="cuda")


@pytest.mark.parametrize("order", [2, 0])
def test_levels_match_oracle(bh, order):
    say(f"[levels] clumpy 50k fp32, target order {order}, {len(LEVELS)} levels")
    pos, mass = inputs.clumpy(50_021, 51)      # ragged last group
    T, p64, m64 = _tree(bh, pos, mass, order=order)
    gl = _levels(len(pos), 1)
    out = T.walk_stats(0.5, 1e-4, theta_levels=(gl, LEVELS))
    acc_f, pot_f = T.forces(0.5, 1e-4, theta_levels=(gl, LEVELS))
    assert torch.equal(acc_f, out["acc"]) and torch.equal(pot_f, out["pot"])
    O = oracle.Tree(p64, m64)
    if order == 2:
        slots = walk_slots(p64, m64)
    else:
        slots = np.empty(len(pos), np.int64)
        slots[O.perm] = np.arange(len(pos))
    th = np.asarray(LEVELS, np.float32).astype(np.float64)[gl.cpu().numpy()[slots // 64]]
    w = O.walk(0.5, 1e-4, theta_per_target=th)
    cnt = out["counts"].cpu().numpy()
    np.testing.assert_array_equal(cnt[:, 0], w["n_pp"])
    np.testing.assert_array_equal(cnt[:, 1], w["n_pc"])
    np.testing.assert_array_equal(out["hash"].cpu().numpy().view(np.uint64), w["hash"])
    check_forces(out["acc"].cpu().numpy(), w["acc"], w["amag"], F32_TOL, "levels", log=say)
    assert pot_err(out["pot"].cpu().numpy(), w["pot"]).max() <= F32_TOL
    T.check()


@pytest.mark.parametrize("case", ["clumpy", "duplicates", "forest"])
def test_levels_equal_per_group_theta(bh, case):
    """The level walk reads S_k precomputed, the per-group walk forms it per step from l and s:
    the same operations, so the same lists and bit-equal results."""
    say(f"[levels] level walk == per-group theta walk: {case}")
    offsets = None
    if case == "clumpy":
        pos, mass = inputs.clumpy(200_000, 52)
    elif case == "duplicates":
        pos, mass = inputs.clumpy(60_000, 53)
        pos[30_000:40_000] = pos[:10_000]      # leaves of several coincident particles
    else:
        rng = np.random.default_rng(54)
        sizes = rng.integers(1, 4000, 30)
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pos = rng.random((offsets[-1], 3)) + np.repeat(rng.random((30, 3)) * 8, sizes, axis=0)
        mass = rng.uniform(0.5, 1.5, offsets[-1])
    T, _, _ = _tree(bh, pos, mass, offsets=offsets)
    gl = _levels(len(pos), 2)
    tg = torch.tensor(np.asarray(LEVELS, np.float32), device="cuda")[gl.long()].contiguous()
    a1 = T.walk_stats(0.5, 1e-4, theta_levels=(gl, LEVELS))
    a2 = T.walk_stats(0.5, 1e-4, theta_group=tg)
    for k in ("acc", "pot", "counts", "hash"):
        assert torch.equal(a1[k], a2[k]), k
    assert torch.equal(a1["group_steps"], a2["group_steps"])


@pytest.mark.parametrize("kind", ["fp64", "order2", "two_per_lane"])
def test_levels_fallback_equals_per_group_theta(bh, kind):
    """Trees the level path does not take (FP64, order 2, two targets per lane) walk the levels'
    values as per-group theta."""
    say(f"[levels] fallback {kind}")
    pos, mass = inputs.clumpy(30_000, 55)
    T, _, _ = _tree(bh, pos, mass, prec="fp64" if kind == "fp64" else "fp32")
    if kind == "order2":
        T.set_order(2)
    if kind == "two_per_lane":
        T.set_walk_config(targets_per_lane=2)
    gl = _levels(len(pos), 3)
    tg = torch.tensor(np.asarray(LEVELS, np.float32), device="cuda")[gl.long()].contiguous()
    a1 = T.walk_stats(0.5, 1e-4, theta_levels=(gl, LEVELS))
    a2 = T.walk_stats(0.5, 1e-4, theta_group=tg)
    for k in ("acc", "pot", "counts", "hash"):
        assert torch.equal(a1[k], a2[k]), k


def test_levels_out_of_range_reported(bh):
    say("[levels] out-of-range level entries")
    pos, mass = inputs.clumpy(20_000, 56)
    T, _, _ = _tree(bh, pos, mass)
    gl = _levels(len(pos), 4, 3)
    bad = gl.clone()
    bad[[2, 9]] = 7                              # beyond the 3 levels given
    a_bad = T.walk_stats(0.5, 1e-4, theta_levels=(bad, LEVELS[:3]))
    with pytest.raises(ValueError, match="theta"):
        T.check()
    fixed = bad.clone()
    fixed[[2, 9]] = 0
    a_ok = T.walk_stats(0.5, 1e-4, theta_levels=(fixed, LEVELS[:3]))
    T.check()
    assert torch.equal(a_bad["hash"], a_ok["hash"]) and torch.equal(a_bad["acc"], a_ok["acc"])


def test_theta_quantize(bh):
    say("[levels] quantisation of per-group theta")
    rng = np.random.default_rng(57)
    th = rng.uniform(0.05, 1.2, 100_001).astype(np.float32)
    th[:4] = [np.nan, np.inf, 0.0, -1.0]
    lv = np.float32([0.1, 0.2, 0.33, 0.5, 0.75, 1.0])
    got = bh.theta_quantize(torch.tensor(th, device="cuda"), list(lv)).cpu().numpy()
    want = np.searchsorted(lv.astype(np.float64), th.astype(np.float64), side="right") - 1
    want = np.where(np.isfinite(th) & (want >= 0), want, 0)
    np.testing.assert_array_equal(got, want)
    # rounding down: every level is at most its theta where that theta is at least the first level
    ok = np.isfinite(th) & (th >= lv[0])
    assert np.all(lv[got[ok]] <= th[ok])


def test_levels_full_size(bh):
    """At the learned benchmark's size (clumpy 4M, FP32, Hilbert walk groups): counts, hashes and
    forces of 2048 sampled targets against the oracle's per-target-theta walk."""
    say("[levels] clumpy4m, 16 levels (sampled targets)")
    pos, mass, spec = inputs.make("clumpy4m")
    lv = list(np.geomspace(0.2, 1.1, 16).astype(np.float32))
    T, p64, m64 = _tree(bh, pos, mass)
    gl = _levels(len(pos), 5, 16)
    out = T.walk_stats(0.5, spec["eps"], theta_levels=(gl, lv))
    idx = inputs.sample_targets(len(pos), 2048, spec["seed"] + 400)
    th = np.asarray(lv, np.float32).astype(np.float64)[gl.cpu().numpy()[walk_slots(p64, m64)[idx] // 64]]
    w = oracle.Tree(p64, m64).walk(0.5, spec["eps"], targets=idx, theta_per_target=th)
    cnt = out["counts"].cpu().numpy()[idx]
    np.testing.assert_array_equal(cnt[:, 0], w["n_pp"])
    np.testing.assert_array_equal(cnt[:, 1], w["n_pc"])
    np.testing.assert_array_equal(out["hash"].cpu().numpy().view(np.uint64)[idx], w["hash"])
    check_forces(out["acc"].cpu().numpy()[idx], w["acc"], w["amag"], F32_TOL, "levels 4M", log=say)
