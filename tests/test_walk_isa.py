"""Guard on the code the compiler makes of the force walk's inner loop (gfx950 assembly of the
FP32 walk, compiled with the library's own flags).

The walk is bound by instruction issue, and its speed has depended on compiler details: the
machine-sinking switch in build.py, the order in which the next record's load and the terms are
scheduled.  This test compiles the FP32 walk to assembly and checks its hottest loop (the
monopole forces walk, scalar node loads, two steps per iteration) for the instruction counts the
step is designed to take: per step 8 vector instructions for the opening test (FP64 offsets, d^2,
two compares) and 12 for the term (r^2 + eps^2 rounded to FP32, v_rsq_f32, three FP32 products,
one conversion, four FP64 sums, the skip update), node records read with scalar loads, no memory
traffic through vector loads or LDS, no scratch, and eight waves per SIMD.
"""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1112_4539_amd import build as libbuild  # noqa: E402

# monopole forces, one target per lane, softened: uniform theta / theta per walk group
MONO = "_ZN2bh6k_walkILb0ELi1ELi0ELb1ELb0EEEvNS_8WalkArgsE"
GROUP = "_ZN2bh6k_walkILb0ELi1ELi0ELb1ELb1EEEvNS_8WalkArgsE"
SRC = "bh_walk_f32.hip"


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    hipcc = libbuild.HIPCC
    if not os.path.exists(hipcc):
        pytest.skip(f"{hipcc} not present")
    out = str(tmp_path_factory.mktemp("isa") / "walk_f32.s")
    flags = [f for f in libbuild.FLAGS if f not in ("-fPIC",)]
    cmd = [hipcc] + flags + libbuild.EXTRA.get(SRC, []) + ["--cuda-device-only", "-S", "-o", out,
                                                           os.path.join(libbuild.CSRC, SRC)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
    return open(out).read().split("\n")


def kernel_lines(lines, name):
    start = next(i for i, l in enumerate(lines) if l.startswith(name + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    meta_end = next(i for i in range(end, len(lines)) if "Occupancy" in lines[i])
    return lines[start:end], lines[end:meta_end + 1]


def inner_loops(body):
    """Instructions of every innermost loop, from the compiler's loop annotations."""
    loops, cur = {}, None
    for i, l in enumerate(body):
        s = l.strip()
        head = re.match(r"^\.LBB(\d+_\d+):", l) or re.match(r"^; %bb\.\d+:", s)
        if head:
            nxt = body[i + 1] if i + 1 < len(body) else ""
            m = re.search(r"in Loop: Header=BB(\d+_\d+)", l)
            if "This Inner Loop Header" in nxt and l.startswith(".LBB"):
                cur = head.group(1)
            elif m:
                cur = m.group(1)
            else:
                cur = None
            continue
        if cur is None or not s or s.startswith(";") or s.startswith("."):
            continue
        loops.setdefault(cur, []).append(s.split()[0])
    return loops


def classify(ops):
    return {
        "valu": sum(1 for o in ops if o.startswith("v_")),
        "rsq": sum(1 for o in ops if o.startswith("v_rsq_f32")),
        "f64": sum(1 for o in ops if o.startswith("v_") and "_f64" in o),
        "smem": sum(1 for o in ops if o.startswith("s_load")),
        "vmem": sum(1 for o in ops if o.startswith(("global_", "flat_", "buffer_", "scratch_"))),
        "lds": sum(1 for o in ops if o.startswith("ds_")),
        "cvt64": sum(1 for o in ops if o.startswith("v_cvt_f64_f32")),
    }


def hot_loops(lines, name):
    body, meta = kernel_lines(lines, name)
    stats = [classify(ops) for ops in inner_loops(body).values()]
    # the scalar-load step loops: two steps (two terms) per iteration, nodes through scalar loads only
    hot = [c for c in stats if c["rsq"] == 2 and c["vmem"] == 0 and c["lds"] == 0 and c["smem"] >= 2]
    return hot, "\n".join(meta)


def test_monopole_walk_loop(asm):
    hot, meta = hot_loops(asm, MONO)
    assert hot, "no scalar-load step loop found in the monopole walk"
    valu = sorted(c["valu"] for c in hot)
    # 2 steps x (8 test + 12 term) vector instructions; the variants for theta > 1 add the
    # particle-range test of the cells that may hold their target
    assert valu[0] <= 40 and valu[-1] <= 44, f"monopole step loops: {valu} VALU per two steps (designed: 40)"
    # one conversion per term (m r^-3 to FP64; the potential takes it too)
    assert all(c["cvt64"] == 2 for c in hot), "a term converts more than m r^-3 to FP64"
    assert all(c["smem"] <= 4 for c in hot), "a step reads its record in more than two scalar loads"
    assert "; ScratchSize: 0" in meta
    occ = int(re.search(r"; Occupancy: (\d+)", meta).group(1))
    assert occ >= 8, f"occupancy {occ} waves per SIMD"


def test_group_theta_walk_loop(asm):
    hot, meta = hot_loops(asm, GROUP)
    assert hot, "no scalar-load step loop found in the per-group-theta walk"
    valu = sorted(c["valu"] for c in hot)
    # the fixed-theta step plus S = fma(l, 1/theta, s)^2 (two FP64 instructions) and a move of s
    # into a vector register (an instruction reads at most one scalar operand, and l and s both
    # come from the scalar record) per step
    assert valu[0] <= 46 and valu[-1] <= 50, f"per-group-theta step loops: {valu} VALU per two steps (designed: 46)"
    # (the record's centre, l, mass and next in two loads, s in a third)
    assert min(c["smem"] for c in hot) <= 6, "the step reads its record in more than three scalar loads"
    assert "; ScratchSize: 0" in meta
