"""GPU neighbour search (the general tree walk of Sec. 4.3, Fig. 4) against the oracle.

Counts and ordered hashes bit-exact (full lists at small n), the SPH density
within 1e-12, in both precisions, in a forest, and at full size on sampled
targets; results independent of the walk order and launch shape.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1112_4539_amd import inputs
from tests.util import tree_cases

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bh():
    import paper_1112_4539_amd as bh
    bh.load()
    assert torch.cuda.is_available()
    return bh


def _gpu(pos, mass, prec):
    dt = torch.float32 if prec == "fp32" else torch.float64
    return torch.tensor(pos, dtype=dt, device="cuda"), torch.tensor(mass, dtype=dt, device="cuda")


def _seen(pos, mass, prec):
    t = np.float32 if prec == "fp32" else np.float64
    return pos.astype(t).astype(np.float64), mass.astype(t).astype(np.float64)


def _compare(bh, pos, mass, prec, radius, targets=None, maxlen=0):
    T = bh.Tree(*_gpu(pos, mass, prec))
    out = T.neighbours(radius, maxlen=maxlen)
    torch.cuda.synchronize()
    O = oracle.Tree(*_seen(pos, mass, prec))
    idx = np.arange(len(pos)) if targets is None else targets
    w = O.neighbours(radius, targets=idx, maxlen=maxlen)
    np.testing.assert_array_equal(out["count"].cpu().numpy()[idx], w["count"])
    np.testing.assert_array_equal(out["hash"].cpu().numpy().view(np.uint64)[idx], w["hash"])
    if maxlen:
        np.testing.assert_array_equal(out["lists"].cpu().numpy()[idx], w["lists"])
    rho = out["rho"].cpu().numpy().astype(np.float64)[idx]
    tol = 1e-12 if prec == "fp64" else 1e-6      # (FP32 output: the density rounded once)
    np.testing.assert_allclose(rho, w["rho"], rtol=tol)
    say(f"  mean neighbours {w['count'].mean():.1f}  max {w['count'].max()}  "
        f"max density rel diff {np.max(np.abs(rho - w['rho']) / w['rho']):.2e}")
    return T, out


@pytest.mark.parametrize("name,radius", [("random1000", 0.1), ("duplicates", 0.4), ("coincident", 0.05),
                                         ("finest_cell_pair", 0.3), ("flat", 0.02), ("random12289", 0.05)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_neighbours_small(bh, name, radius, prec):
    say(f"[nbr] case={name} radius={radius} {prec}")
    pos = tree_cases()[name]
    mass = np.random.default_rng(len(pos)).random(len(pos)) + 0.5
    _compare(bh, pos, mass, prec, radius, maxlen=len(pos))


@pytest.mark.parametrize("name,radius", [("duplicates", 0.4), ("coincident", 0.05), ("finest_cell_pair", 0.3)])
def test_neighbours_subnormal_fp32(bh, name, radius):
    """Leaves of several particles (coincident Morton keys) read each particle's FP32 position and
    mass and widen them to FP64: subnormal FP32 coordinates (the case scaled by 1e-39, counts,
    hashes and lists only, as the density overflows FP32 there) and subnormal FP32 masses (the
    density checked)."""
    say(f"[nbr] case={name} fp32 subnormal coordinates, then subnormal masses")
    pos = tree_cases()[name]
    rng = np.random.default_rng(len(pos) + 7)
    mass = rng.random(len(pos)) + 0.5
    tiny = (pos * 1e-39).astype(np.float32)
    assert np.any((tiny != 0) & (np.abs(tiny) < np.finfo(np.float32).tiny))
    T = bh.Tree(*_gpu(tiny, mass, "fp32"))
    out = T.neighbours(radius * 1e-39, maxlen=len(pos), density=False)
    torch.cuda.synchronize()
    w = oracle.Tree(*_seen(tiny, mass, "fp32")).neighbours(radius * 1e-39, maxlen=len(pos))
    assert w["count"].sum() > 0
    np.testing.assert_array_equal(out["count"].cpu().numpy(), w["count"])
    np.testing.assert_array_equal(out["hash"].cpu().numpy().view(np.uint64), w["hash"])
    np.testing.assert_array_equal(out["lists"].cpu().numpy(), w["lists"])
    small = (mass * 1e-39).astype(np.float32)
    assert np.all(small < np.finfo(np.float32).tiny)
    _compare(bh, pos, small, "fp32", radius, maxlen=len(pos))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_neighbours_clumpy_and_orders(bh, prec):
    say(f"[nbr] clumpy 100k radius 0.005 {prec}, every target order and launch shape")
    pos, mass = inputs.clumpy(100_000, 19)
    T, ref = _compare(bh, pos, mass, prec, 0.005, maxlen=64)
    for order in (0, 1, 2):
        for chunk in (0, 8, -1):
            T.set_walk_config(xcd_chunk=chunk, target_order=order)
            out = T.neighbours(0.005, maxlen=64)
            for k in ("count", "hash", "lists", "rho"):
                assert torch.equal(out[k], ref[k]), (order, chunk, k)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_neighbours_full_size_sampled(bh, prec):
    """The benchmarked search (clumpy 4M, r = 2e-3, the launch bench.py times) on sampled targets."""
    say(f"[nbr] clumpy4m radius 2e-3 {prec} (sampled targets)")
    pos, mass, spec = inputs.make("clumpy4m")
    tg = inputs.sample_targets(len(pos), 2048, 77)
    _compare(bh, pos, mass, prec, 2e-3, targets=tg)


def test_neighbours_forest(bh):
    say("[nbr] forest of 40 clusters: each cluster's neighbours equal its own tree's")
    pos, mass, off = inputs.clusters(40, 11, nmin=100, nmax=3000)
    gp, gm = _gpu(pos, mass, "fp32")
    F = bh.build_forest(gp, gm, torch.tensor(off, device="cuda"))
    out = F.neighbours(0.3, maxlen=32)
    torch.cuda.synchronize()
    for k in range(len(off) - 1):
        b, e = int(off[k]), int(off[k + 1])
        T = bh.Tree(gp[b:e].contiguous(), gm[b:e].contiguous())
        one = T.neighbours(0.3, maxlen=32)
        for key in ("count", "hash", "lists", "rho"):
            assert torch.equal(out[key][b:e], one[key]), (k, key)


def test_neighbours_bad_radius(bh):
    pos = torch.rand((100, 3), device="cuda")
    T = bh.Tree(pos, torch.ones(100, device="cuda"))
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            T.neighbours(bad)
