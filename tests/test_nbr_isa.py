"""Guard on the code the compiler makes of the neighbour walk (gfx950 assembly of bh_nbr.hip,
compiled with the library's own flags).

The walk's speed rests on its node records and group particles being read with wave-uniform
scalar loads, one batch per round trip, and has depended on compiler details: a change of
structure once made the compiler treat the cursor as divergent and read every record with
vector loads.  This test compiles the file to assembly and checks the FP32 search without lists
(the one bench.py times): no vector memory access inside the walk's loops (only the per-target
setup, the per-cluster bounds and the results use vector memory), the record read with a 32-bit
offset in a scalar register, no scratch, and eight waves per SIMD.
"""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1112_4539_amd import build as libbuild  # noqa: E402

KERNEL = "_ZN2bh12_GLOBAL__N_15k_nbrILb0ELb0EEEvNS0_7NbrArgsE"
SRC = "bh_nbr.hip"
VMEM = ("global_", "flat_", "buffer_", "scratch_")


@pytest.fixture(scope="module")
def body():
    hipcc = libbuild.HIPCC
    if not os.path.exists(hipcc):
        pytest.skip(f"{hipcc} not present")
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "nbr.s")
        flags = [f for f in libbuild.FLAGS if f not in ("-fPIC",)]
        cmd = [hipcc] + flags + libbuild.EXTRA.get(SRC, []) + ["--cuda-device-only", "-S", "-o", out,
                                                               os.path.join(libbuild.CSRC, SRC)]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, r.stdout[-2000:]
        lines = open(out).read().split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(KERNEL + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    meta_end = next(i for i in range(end, len(lines)) if "Occupancy" in lines[i])
    return lines[start:end], lines[end:meta_end + 1]


def by_depth(code):
    """(loop depth, instruction) for every instruction, from the compiler's loop annotations."""
    out, depth = [], 0
    for i, l in enumerate(code):
        s = l.strip()
        if re.match(r"^(\.LBB\d+_\d+:|; %bb\.\d+:)", s):
            nxt = code[i + 1].strip() if i + 1 < len(code) else ""
            # a loop header's own depth is on the line after its label ("This Loop Header:
            # Depth=N"); the label line of a header names its parent loop instead
            m = re.search(r"Loop Header: Depth=(\d+)", nxt) or re.search(r"in Loop: Header=\S+ Depth=(\d+)", l)
            depth = int(m.group(1)) if m else 0
            continue
        if not s or s.startswith(";") or s.startswith("."):
            continue
        out.append((depth, s))
    return out


def test_walk_loops_use_scalar_memory_only(body):
    code, _ = body
    ins = by_depth(code)
    assert any(d >= 2 for d, _ in ins), "no nested loops found: the annotations changed"
    vmem = [s for d, s in ins if d >= 2 and s.split()[0].startswith(VMEM)]
    assert not vmem, f"vector memory inside the walk's loops: {vmem[:5]}"
    smem = [s for d, s in ins if d >= 2 and s.startswith("s_load")]
    assert smem, "no scalar loads inside the walk's loops"


def test_record_load_takes_a_32bit_offset(body):
    code, _ = body
    ins = by_depth(code)
    # the 64-byte record: its first 32 bytes in one s_load_dwordx8 at an SGPR byte offset
    pat = re.compile(r"^s_load_dwordx8 s\[\d+:\d+\], s\[\d+:\d+\], s\d+ offset:0x0$")
    assert any(d >= 2 and pat.match(s) for d, s in ins)


def test_no_scratch_eight_waves(body):
    _, meta = body
    text = "\n".join(meta)
    assert re.search(r"; ScratchSize: 0\b", text)
    occ = int(re.search(r"; Occupancy: (\d+)", text).group(1))
    assert occ >= 8
