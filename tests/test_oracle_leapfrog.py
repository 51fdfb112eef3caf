"""Pins of the oracle's time loop (Sec. 1: force, integrate, repeat) -- the kick-drift-kick
leapfrog on the direct-sum forces -- against Kepler's two-body problem."""
import math

import numpy as np
import pytest


def _binary(e, m1=0.6, m2=0.4, a=1.0):
    """Two bodies on a Kepler orbit of semi-major axis a and eccentricity e, started at pericentre,
    centre of mass at rest at the origin.  Returns pos, vel, mass, period, energy, angular momentum."""
    M = m1 + m2
    rp = a * (1 - e)
    vp = math.sqrt(M * (1 + e) / (a * (1 - e)))      # vis-viva at pericentre, G = 1
    pos = np.array([[rp * m2 / M, 0.0, 0.0], [-rp * m1 / M, 0.0, 0.0]])
    vel = np.array([[0.0, vp * m2 / M, 0.0], [0.0, -vp * m1 / M, 0.0]])
    P = 2 * math.pi * math.sqrt(a ** 3 / M)
    E = -m1 * m2 / (2 * a)
    Lz = m1 * m2 / M * rp * vp
    return pos, vel, np.array([m1, m2]), P, E, Lz


def _energy(pos, vel, mass, pot):
    return 0.5 * np.sum(mass * np.sum(vel * vel, axis=1)) + 0.5 * np.sum(mass * pot)


def _lz(pos, vel, mass):
    return np.sum(mass * (pos[:, 0] * vel[:, 1] - pos[:, 1] * vel[:, 0]))


@pytest.mark.parametrize("e", [0.0, 0.5])
def test_kepler_period_energy_and_angular_momentum(oracle_mod, e):
    pos, vel, mass, P, E, Lz = _binary(e)
    steps = 4000
    dt = P / steps
    p1, v1, a1, pot1 = oracle_mod.leapfrog(pos, vel, mass, 0.0, dt, steps)
    # after one period the bodies are back at pericentre (second-order phase error)
    sep0 = pos[0] - pos[1]
    sep1 = p1[0] - p1[1]
    assert np.linalg.norm(sep1 - sep0) < (3e-4 if e else 1e-5)
    # energy: the leapfrog's error is bounded and second order, angular momentum exact to rounding
    assert abs(_energy(p1, v1, mass, pot1) / E - 1) < (2e-4 if e else 1e-6)
    assert abs(_lz(p1, v1, mass) / Lz - 1) < 1e-12
    # momentum stays zero (the pair forces are equal and opposite)
    assert np.linalg.norm((mass[:, None] * v1).sum(0)) < 1e-14


def test_leapfrog_second_order(oracle_mod):
    pos, vel, mass, P, E, Lz = _binary(0.3)
    errs = []
    for steps in (500, 1000, 2000):
        p1, v1, _, _ = oracle_mod.leapfrog(pos, vel, mass, 0.0, 0.25 * P / steps, steps)
        errs.append(p1)
    ref = oracle_mod.leapfrog(pos, vel, mass, 0.0, 0.25 * P / 8000, 8000)[0]
    e = [np.linalg.norm(x - ref) for x in errs]
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5


def test_leapfrog_time_reversible(oracle_mod):
    rng = np.random.default_rng(2)
    pos = rng.normal(size=(20, 3))
    vel = 0.1 * rng.normal(size=(20, 3))
    mass = rng.random(20) + 0.5
    p1, v1, a1, _ = oracle_mod.leapfrog(pos, vel, mass, 0.1, 0.01, 200)
    p0, v0, _, _ = oracle_mod.leapfrog(p1, -v1, mass, 0.1, 0.01, 200, acc=a1)
    np.testing.assert_allclose(p0, pos, atol=1e-10)
    np.testing.assert_allclose(-v0, vel, atol=1e-10)
