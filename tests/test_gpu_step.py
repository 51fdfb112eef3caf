"""GPU time loop (Sec. 1: forces, orbit integration, repeat): the leapfrog step against the
oracle's leapfrog on the direct sum, and the Morton reorder against the plain order."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1112_4539_amd import inputs

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


def _state(bh, pos, vel, mass, dt_, theta, eps):
    d = torch.device("cuda")
    P = torch.tensor(pos, dtype=dt_, device=d)
    V = torch.tensor(vel, dtype=dt_, device=d)
    M = torch.tensor(mass, dtype=dt_, device=d)
    A, U = bh.Tree(P, M).forces(theta, eps)
    return P, V, M, A.clone(), U.clone()


def test_kepler_two_body_matches_oracle(bh):
    say("[step] Kepler e=0.5, FP64, 2000 steps")
    m1, m2, a, e = 0.6, 0.4, 1.0, 0.5
    M = m1 + m2
    rp = a * (1 - e)
    vp = math.sqrt(M * (1 + e) / (a * (1 - e)))
    pos = np.array([[rp * m2 / M, 0.0, 0.0], [-rp * m1 / M, 0.0, 0.0]])
    vel = np.array([[0.0, vp * m2 / M, 0.0], [0.0, -vp * m1 / M, 0.0]])
    mass = np.array([m1, m2])
    Pd = 2 * math.pi * math.sqrt(a ** 3 / M)
    dt, steps = Pd / 2000, 2000
    P, V, Mt, A, U = _state(bh, pos, vel, mass, torch.float64, 0.5, 0.0)
    ws = None
    for _ in range(steps):
        ws = bh.leapfrog_step(P, V, Mt, A, U, dt, 0.5, 0.0, workspace=ws)
    torch.cuda.synchronize()
    po, vo, ao, uo = oracle.leapfrog(pos, vel, mass, 0.0, dt, steps)
    np.testing.assert_allclose(P.cpu().numpy(), po, rtol=0, atol=1e-12)
    np.testing.assert_allclose(V.cpu().numpy(), vo, rtol=0, atol=1e-12)
    sep = P.cpu().numpy()[0] - P.cpu().numpy()[1]
    # back at pericentre after one period, up to the leapfrog's second-order phase error
    assert np.linalg.norm(sep - (pos[0] - pos[1])) < 2e-3


def test_plummer_steps_match_oracle_at_tiny_theta(bh):
    say("[step] Plummer 2k FP64, theta 1e-7 (every term a particle term), 20 steps")
    pos, mass = inputs.plummer(2048, 21)
    rng = np.random.default_rng(5)
    vel = 0.3 * rng.normal(size=pos.shape)
    # (theta 1e-7: a cell of side l could only be accepted beyond l / theta, more than 100 times the
    # smallest side of 2^-21 of the root cube: farther than any particle)
    P, V, Mt, A, U = _state(bh, pos, vel, mass, torch.float64, 1e-7, 0.01)
    ws = None
    for _ in range(20):
        ws = bh.leapfrog_step(P, V, Mt, A, U, 1e-3, 1e-7, 0.01, workspace=ws)
    torch.cuda.synchronize()
    po, vo, ao, uo = oracle.leapfrog(pos, vel, mass, 0.01, 1e-3, 20)
    # the walk sums in depth-first order, the oracle in index order: rounding-level differences per
    # force, grown over 20 steps by close encounters
    assert np.abs(P.cpu().numpy() - po).max() < 1e-11
    assert np.abs(V.cpu().numpy() - vo).max() < 1e-9
    assert np.max(np.abs(U.cpu().numpy() - uo) / np.abs(uo)) < 1e-11


@pytest.mark.parametrize("prec,order", [("fp32", 1), ("fp32", 2), ("fp64", 1)])
def test_reorder_is_a_permutation_of_the_plain_loop(bh, prec, order):
    say(f"[step] clumpy 20k {prec} order {order}: 5 steps with and without the Morton reorder")
    pos, mass = inputs.clumpy(20_000, 23)
    vel = 0.1 * np.random.default_rng(6).normal(size=pos.shape)
    dt_ = torch.float32 if prec == "fp32" else torch.float64
    runs = []
    for reorder in (False, True):
        P, V, Mt, A, U = _state(bh, pos, vel, mass, dt_, 0.5, 1e-4)
        ids = torch.arange(len(pos), dtype=torch.int64, device="cuda")
        ws = None
        for _ in range(5):
            ws = bh.leapfrog_step(P, V, Mt, A, U, 2e-4, 0.5, 1e-4, order=order, reorder=reorder, ids=ids,
                                  workspace=ws)
        torch.cuda.synchronize()
        inv = torch.empty_like(ids)
        inv[ids] = torch.arange(len(pos), dtype=torch.int64, device="cuda")
        runs.append([x[inv] for x in (P, V, Mt, A, U)])
        if reorder:
            assert not torch.equal(ids, torch.arange(len(pos), device="cuda"))
            assert torch.equal(torch.sort(ids).values, torch.arange(len(pos), device="cuda"))
    for x, y in zip(*runs):
        assert torch.equal(x, y)


def test_energy_conservation(bh):
    say("[step] Plummer 4k FP64 theta 0.4, 100 steps: energy drift")
    pos, mass = inputs.plummer(4096, 24)
    # velocities of a cold collapse would not conserve well with a fixed step; take a small random field
    vel = 0.05 * np.random.default_rng(7).normal(size=pos.shape)
    P, V, Mt, A, U = _state(bh, pos, vel, mass, torch.float64, 0.4, 0.05)

    def energy():
        return float(0.5 * (Mt * (V * V).sum(1)).sum() + 0.5 * (Mt * U).sum())

    E0 = energy()
    ws = None
    for _ in range(100):
        ws = bh.leapfrog_step(P, V, Mt, A, U, 2e-3, 0.4, 0.05, reorder=True, workspace=ws)
    torch.cuda.synchronize()
    say(f"  E0 {E0:.9f} E {energy():.9f} rel {abs(energy() / E0 - 1):.2e}")
    # (tree forces at theta 0.4 are not exact gradients: measured drift 1.6e-5 over the 100 steps)
    assert abs(energy() / E0 - 1) < 1e-4
