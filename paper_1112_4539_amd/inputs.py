"""Seeded synthetic particle sets shared by the tests, the smoke check and the bench.

This module holds input generation only (random draws and the closed-form
inverse CDF of the Plummer mass profile); none of the force method's
arithmetic lives here.  All draws use ``numpy.random.default_rng`` in float64,
in the order documented on each function, so any consumer regenerates the same
particles from the same seed.

Workloads (stand-ins for the uniform sphere, cube and disk-galaxy sets of the
paper's Sec. 5; no dataset is read):

* ``plummer``  -- Plummer sphere, scale radius a, truncated at r < R = 10a,
  equal masses summing to M.
* ``clumpy``   -- 25% uniform in the unit cube plus 75% split evenly over 64
  Plummer sub-clusters (a = 0.01, R = 0.1) centred uniformly in the cube.
* ``clusters`` -- K independent Plummer clusters with log-uniform sizes.
"""
from __future__ import annotations

import numpy as np


def plummer_mass_fraction(r, a=1.0):
    """Mass inside radius r of an untruncated Plummer sphere of unit mass."""
    r = np.asarray(r, np.float64)
    return r ** 3 / (r * r + a * a) ** 1.5


def _plummer_from_uniforms(u, v, w, a, rmax, mtot):
    """Map three uniform draws per particle to a truncated Plummer sphere.

    Radius by the inverse CDF of the truncated mass profile:
    X = u * M(rmax), r = a / sqrt(X^(-2/3) - 1); direction isotropic with
    cos(polar) = 2v - 1 and azimuth 2*pi*w.
    """
    n = u.shape[0]
    mfrac = float(plummer_mass_fraction(rmax / a, 1.0))
    X = u * mfrac
    with np.errstate(divide="ignore"):
        r = a / np.sqrt(np.power(X, -2.0 / 3.0) - 1.0)
    r = np.where(X > 0, r, 0.0)
    ct = 2.0 * v - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * w
    pos = np.empty((n, 3))
    pos[:, 0] = r * st * np.cos(ph)
    pos[:, 1] = r * st * np.sin(ph)
    pos[:, 2] = r * ct
    mass = np.full(n, mtot / n)
    return pos, mass


def plummer(n, seed, a=1.0, rmax=10.0, mtot=1.0, rng=None):
    """Truncated Plummer sphere (float64).  Draw order: u, v, w = rng.random(n) x3."""
    rng = np.random.default_rng(seed) if rng is None else rng
    u = rng.random(n)
    v = rng.random(n)
    w = rng.random(n)
    return _plummer_from_uniforms(u, v, w, a, rmax, mtot)


def clumpy(n, seed, n_clumps=64, uniform_frac=0.25, a=0.01, rmax=0.1):
    """Clumpy field (float64): uniform background plus equal-mass Plummer clumps.

    Draw order: centres = rng.random((n_clumps, 3)); background =
    rng.random((n_uniform, 3)); then each clump in centre order draws its
    Plummer uniforms (u, v, w).  Every particle has mass 1/n.
    """
    rng = np.random.default_rng(seed)
    n_uni = int(round(n * uniform_frac))
    per = (n - n_uni) // n_clumps
    n_uni = n - per * n_clumps
    centres = rng.random((n_clumps, 3))
    parts = [rng.random((n_uni, 3))]
    for c in range(n_clumps):
        p, _ = plummer(per, None, a=a, rmax=rmax, mtot=1.0, rng=rng)
        parts.append(p + centres[c])
    pos = np.concatenate(parts, axis=0)
    mass = np.full(n, 1.0 / n)
    return pos, mass


def cluster_sizes(k, seed, nmin=1024, nmax=65536):
    """Log-uniform cluster sizes floor(exp(U(ln nmin, ln nmax))), drawn first from the stream."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=k))).astype(np.int64)
    return sizes, rng


def clusters(k, seed, nmin=1024, nmax=65536, a=1.0, rmax=10.0, mtot=1.0):
    """K independent Plummer clusters, concatenated; returns (pos, mass, offsets[k+1])."""
    sizes, rng = cluster_sizes(k, seed, nmin, nmax)
    pos, mass = [], []
    for nk in sizes:
        p, m = plummer(int(nk), None, a=a, rmax=rmax, mtot=mtot, rng=rng)
        pos.append(p)
        mass.append(m)
    offsets = np.zeros(k + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    return np.concatenate(pos), np.concatenate(mass), offsets


def sample_targets(n, count, seed):
    """Sorted sample of ``count`` distinct particle indices, from default_rng([seed, 1])."""
    count = min(count, n)
    rng = np.random.default_rng([seed, 1])
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


# Named workloads: (generator, kwargs, softening, theta list, precision)
WORKLOADS = {
    "plummer4k": dict(kind="plummer", n=4096, seed=0, eps=0.01, thetas=(0.5,), prec="fp64"),
    "plummer1m": dict(kind="plummer", n=1048576, seed=1, eps=0.005, thetas=(0.3, 0.5, 0.75), prec="fp32"),
    "clumpy4m": dict(kind="clumpy", n=4194304, seed=2, eps=1e-4, thetas=(0.5,), prec="fp32"),
    "clumpy8m": dict(kind="clumpy", n=8388608, seed=4, eps=1e-4, thetas=(0.5,), prec="fp32"),
}


def make(name):
    """Generate a named workload; returns (pos float64 [n,3], mass float64 [n], spec)."""
    spec = WORKLOADS[name]
    if spec["kind"] == "plummer":
        pos, mass = plummer(spec["n"], spec["seed"])
    else:
        pos, mass = clumpy(spec["n"], spec["seed"])
    return pos, mass, spec
