"""CPU-side checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here (there is no GPU in the build container); the
argument checks that fail before any device work are exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bh.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("bh_build_tree", "bh_forces", "bh_forces_theta", "bh_direct", "bh_workspace_bytes",
                 "bh_walk_stats", "bh_tree_export", "bh_tree_release", "bh_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1112_4539_amd as bh
    lib = bh.load()
    for name in _declared():
        assert hasattr(lib, name), name
    # nothing else with C linkage leaks out under the bh_ prefix
    out = os.popen(f"nm -D --defined-only {bh.LIB_PATH}").read()
    exported = sorted(set(re.findall(r"\s(bh_[a-z_0-9]+)$", out, flags=re.M)))
    assert exported == _declared()


def test_host_side_argument_checks():
    import paper_1112_4539_amd as bh
    lib = bh.load()
    assert lib.bh_version() == 3
    assert lib.bh_workspace_bytes(-1, 0) == -1
    assert lib.bh_workspace_bytes(1 << 31, 0) == -1
    assert lib.bh_workspace_bytes(1 << 30, 0) == -1          # indices are 32-bit: n <= 2^30 - 1
    assert lib.bh_workspace_bytes((1 << 30) - 1, 0) > 0
    assert lib.bh_workspace_bytes(10, 7) == -1
    w1 = lib.bh_workspace_bytes(1000, 0)
    w2 = lib.bh_workspace_bytes(1000, 1)
    assert 0 < w1 < w2
    assert lib.bh_workspace_bytes(2000, 0) > w1
    out = ctypes.c_void_p()
    # bad precision / n / missing workspace are rejected before any GPU work
    assert lib.bh_build_tree(None, None, 10, 5, None, 0, None, ctypes.byref(out)) == -1
    assert lib.bh_build_tree(None, None, -3, 0, None, 0, None, ctypes.byref(out)) == -1
    assert lib.bh_build_tree(ctypes.c_void_p(256), ctypes.c_void_p(512), 10, 0, None, 0, None,
                             ctypes.byref(out)) == -2
    assert b"workspace" in lib.bh_last_error()
    assert lib.bh_forces(None, 0.5, 0.01, None, None, None) == -1
    assert lib.bh_direct(None, None, 10, 0, None, 5, -1.0, None, None, None) == -1
    assert lib.bh_set_walk_config(None, 4, 0, 0, 0, 0, 1) == -1
    out = ctypes.c_void_p()
    assert lib.bh_build_forest(None, None, None, 2, 10, 0, None, 0, None, ctypes.byref(out)) == -1
    assert lib.bh_forest_workspace_bytes(10, 0, 0) == -1
    assert lib.bh_forest_workspace_bytes(10, 1, 0) == lib.bh_workspace_bytes(10, 0)
    assert lib.bh_forest_workspace_bytes(10, 512, 0) > lib.bh_workspace_bytes(10, 0)
    assert lib.bh_graph_launch(None, None) == -1
    n_param, n_grad, n_wb, n_part = (ctypes.c_int64() for _ in range(4))
    assert lib.bh_mlp_sizes(4096, ctypes.byref(n_param), ctypes.byref(n_grad), ctypes.byref(n_wb),
                            ctypes.byref(n_part)) == 0
    assert (n_param.value, n_grad.value, n_wb.value) == (4801, 4802, 8768)
    assert n_part.value == 128 * 4802
    assert lib.bh_mlp_infer(None, None, None, None, 10, ctypes.c_float(1.0), ctypes.c_float(0.5), None, None) == -1
    assert lib.bh_autotune(None, 0.5, 0.0, None, None, 1, None, None, None, 0, None) == -1


def test_theta_bound_matches_header():
    import paper_1112_4539_amd as bh
    assert abs(bh.THETA_MAX - 2 / 3 ** 0.5) < 1e-15
