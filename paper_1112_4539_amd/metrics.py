"""Force-error statistics of a walk against a reference (measurement, not the method).

Sec. 5, Eq. (4) measures the accuracy of the tree forces by the mean over
particles of |a_tree - a_ref| / |a_ref|; the headline figure here is the RMS of
the same per-particle relative error.  Both work on torch tensors on any device
(the benchmark keeps them on the GPU), accumulate in float64, and skip nothing:
a reference force of exactly zero has no relative error and is rejected.
"""
from __future__ import annotations

import torch


def rel_errors(acc, acc_ref):
    """Per-particle |acc_i - acc_ref_i| / |acc_ref_i| (float64), both [m, 3]."""
    a = torch.as_tensor(acc).to(torch.float64)
    r = torch.as_tensor(acc_ref).to(device=a.device, dtype=torch.float64)
    if a.shape != r.shape or a.dim() != 2 or a.shape[1] != 3:
        raise ValueError("acc and acc_ref must both be [m, 3]")
    den = torch.linalg.vector_norm(r, dim=1)
    if bool((den == 0).any()):
        raise ValueError("a reference acceleration of exactly zero has no relative error")
    return torch.linalg.vector_norm(a - r, dim=1) / den


def rms_rel_err(acc, acc_ref):
    """sqrt(mean_i (|acc_i - acc_ref_i| / |acc_ref_i|)^2): the RMS form of Eq. (4)."""
    e = rel_errors(acc, acc_ref)
    return float(torch.sqrt(torch.mean(e * e)).item())


def mean_rel_err(acc, acc_ref):
    """mean_i |acc_i - acc_ref_i| / |acc_ref_i|: Eq. (4)."""
    return float(torch.mean(rel_errors(acc, acc_ref)).item())
