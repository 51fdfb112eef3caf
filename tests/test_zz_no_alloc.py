"""The allocation-free entry point (bh_forces_noalloc) against bh_build_tree + bh_forces.

It runs the same kernels on the library's static scratch array instead of a
workspace, so its results must equal the workspace path's bit for bit; two
calls in a row (the second smaller) check that the array keeps no state that
matters, and sizes past the stated maximum are rejected.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1112_4539_amd import inputs
from tests.util import check_forces

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


def _noalloc(bh, pos, mass, theta, eps):
    lib = bh.load()
    n = pos.shape[0]
    acc = torch.full((n, 3), float("nan"), dtype=pos.dtype, device=pos.device)
    pot = torch.full((n,), float("nan"), dtype=pos.dtype, device=pos.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.bh_forces_noalloc(ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(mass.data_ptr()), n,
                               0 if pos.dtype == torch.float32 else 1, theta, eps, ctypes.c_void_p(acc.data_ptr()),
                               ctypes.c_void_p(pot.data_ptr()), st)
    assert rc == 0, lib.bh_last_error()
    torch.cuda.synchronize()
    return acc, pot


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_workspace_path(bh, prec):
    dt = torch.float32 if prec == "fp32" else torch.float64
    # first the largest size it takes, then a smaller ragged one, then a tiny one
    cases = [("clumpy", bh.NOALLOC_MAX_N, 0.5, 1e-4, 61), ("plummer", 12_345, 0.6, 0.01, 62),
             ("plummer", 3, 0.5, 0.01, 63)]
    for kind, n, theta, eps, seed in cases:
        say(f"[noalloc] {prec} {kind} n={n} theta={theta}")
        pos, mass = (inputs.clumpy(n, seed) if kind == "clumpy" else inputs.plummer(n, seed))
        gp = torch.tensor(pos, dtype=dt, device="cuda")
        gm = torch.tensor(mass, dtype=dt, device="cuda")
        a0, p0 = _noalloc(bh, gp, gm, theta, eps)
        T = bh.Tree(gp, gm)
        a1, p1 = T.forces(theta, eps)
        torch.cuda.synchronize()
        assert torch.equal(a0, a1) and torch.equal(p0, p1), (kind, n)
        if n <= 20_000:
            p64 = pos.astype(np.float32 if prec == "fp32" else np.float64).astype(np.float64)
            m64 = mass.astype(np.float32 if prec == "fp32" else np.float64).astype(np.float64)
            w = oracle.Tree(p64, m64).walk(theta, eps)
            check_forces(a0.cpu().numpy(), w["acc"], w["amag"], 1e-5 if prec == "fp32" else 1e-12, "noalloc",
                         log=say)


def test_noalloc_rejects_beyond_maximum(bh):
    lib = bh.load()
    n = bh.NOALLOC_MAX_N + 1
    gp = torch.rand((n, 3), device="cuda")
    gm = torch.ones(n, device="cuda")
    acc = torch.empty((n, 3), device="cuda")
    pot = torch.empty((n,), device="cuda")
    rc = lib.bh_forces_noalloc(ctypes.c_void_p(gp.data_ptr()), ctypes.c_void_p(gm.data_ptr()), n, 0, 0.5, 0.01,
                               ctypes.c_void_p(acc.data_ptr()), ctypes.c_void_p(pot.data_ptr()), None)
    assert rc == -1 and b"bh_forces_noalloc" in lib.bh_last_error()
    with pytest.raises(ValueError):
        bh.forces_noalloc(gp, gm, 0.5, 0.01, acc, pot)
    # the Python wrapper takes caller-owned outputs and calls the same entry point
    m = 5000
    a, p = bh.forces_noalloc(gp[:m].contiguous(), gm[:m].contiguous(), 0.5, 0.01, acc[:m], pot[:m])
    T = bh.Tree(gp[:m].contiguous(), gm[:m].contiguous())
    a1, p1 = T.forces(0.5, 0.01)
    assert torch.equal(a, a1) and torch.equal(p, p1)
