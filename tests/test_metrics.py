"""Pins of the force-error statistics (Sec. 5, Eq. (4) and its RMS form).

Both the oracle's numpy versions and the package's torch versions (used by
the benchmark and the learned-theta code) are checked against errors built
by hand, with per-particle relative errors chosen so that the mean and the
RMS differ, and the direction and scale of each error vary.
"""
import math

import numpy as np
import pytest
import torch

from paper_1112_4539_amd import metrics


def _constructed(rel, seed):
    """acc_ref with random directions and magnitudes over six decades; acc = acc_ref plus an error
    of exactly |acc_ref_i| * rel_i in a random direction."""
    rng = np.random.default_rng(seed)
    m = len(rel)
    ref = rng.normal(size=(m, 3))
    ref *= (10.0 ** rng.uniform(-3, 3, m) / np.linalg.norm(ref, axis=1))[:, None]
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    acc = ref + u * (np.linalg.norm(ref, axis=1) * np.asarray(rel))[:, None]
    return acc, ref


REL = [0.1, 0.3, 0.0, 0.4, 2e-3, 0.05]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_statistics_on_constructed_errors(oracle_mod, seed):
    acc, ref = _constructed(REL, seed)
    mean = math.fsum(REL) / len(REL)
    rms = math.sqrt(math.fsum(r * r for r in REL) / len(REL))
    assert abs(oracle_mod.mean_rel_err(acc, ref) - mean) <= 1e-12
    assert abs(oracle_mod.rms_rel_err(acc, ref) - rms) <= 1e-12
    # the two statistics are not interchangeable on these errors
    assert abs(mean - rms) > 0.05


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_package_statistics_on_constructed_errors(seed):
    acc, ref = _constructed(REL, seed)
    mean = math.fsum(REL) / len(REL)
    rms = math.sqrt(math.fsum(r * r for r in REL) / len(REL))
    for dt in (torch.float64, torch.float32):
        a = torch.tensor(acc, dtype=dt)
        # (float32 input: acc rounded to float32 first, relative error 2^-24 of |acc_i|)
        tol = 1e-12 if dt == torch.float64 else 1e-6
        assert abs(metrics.mean_rel_err(a, ref) - mean) <= tol
        assert abs(metrics.rms_rel_err(a, torch.tensor(ref)) - rms) <= tol
        e = metrics.rel_errors(a, torch.tensor(ref)).numpy()
        np.testing.assert_allclose(e, REL, atol=3 * tol)


def test_statistics_ignore_particle_order_and_scale():
    acc, ref = _constructed(REL, 5)
    p = np.random.default_rng(9).permutation(len(REL))
    s = 2.0 ** 37
    assert metrics.rms_rel_err(torch.tensor(acc[p] * s), torch.tensor(ref[p] * s)) == pytest.approx(
        metrics.rms_rel_err(torch.tensor(acc), torch.tensor(ref)), rel=1e-14)


def test_zero_reference_rejected():
    ref = np.array([[1.0, 0, 0], [0.0, 0.0, 0.0]])
    with pytest.raises(ValueError):
        metrics.rms_rel_err(torch.tensor(ref), torch.tensor(ref))
    with pytest.raises(ValueError):
        metrics.rel_errors(torch.zeros(3, 2), torch.zeros(3, 2))
