"""CPU FP64 oracle for the Barnes-Hut tree method (arXiv:1112.4539).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the GPU library never
does, and this package imports nothing from it.

The arithmetic lives in ``bh_oracle.c`` (plain C, binary64, no FP contraction);
this module only loads it and marshals numpy arrays.  Definitions followed:

* ``direct``      -- Sec. 3, Eq. (1): softened pair sum over j != i.  The
  acceleration is attractive, the potential is the physical ``-sum m/r``.
* ``Tree``        -- Sec. 4.1 recursive oct-tree on the 2^21 grid of the root
  cube, compressed, with the Sec. 4.4 monopole moments and Eq. (2) cell sizes.
* ``Tree.walk``   -- Fig. 3 recursive walk with the opening test of Eq. (2)/(3);
  ``order=2`` adds the quadrupole cell term (Sec. 4.1, Sec. 7: higher moments).
* ``Tree.neighbours`` -- Sec. 4.3, Fig. 4: the general tree walk as a neighbour
  search with the SPH density as its per-neighbour work.
* ``leapfrog``    -- Sec. 1: the time loop (forces, orbit integration, repeat), as the
  kick-drift-kick leapfrog on the direct-sum forces.
* ``rms_rel_err`` / ``mean_rel_err`` -- Sec. 5, Eq. (4) and its RMS form.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``bh_oracle.c`` into ``liboracle.so`` with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    d = ctypes.c_double
    lib.orc_direct.argtypes = [P, P, i64, P, i64, d, P, P, P]
    lib.orc_direct.restype = ctypes.c_int
    lib.orc_tree_build.argtypes = [P, P, i64]
    lib.orc_tree_build.restype = P
    lib.orc_tree_free.argtypes = [P]
    lib.orc_tree_free.restype = None
    lib.orc_tree_nodes.argtypes = [P]
    lib.orc_tree_nodes.restype = i64
    lib.orc_tree_cube.argtypes = [P, P, P]
    lib.orc_tree_cube.restype = None
    lib.orc_tree_export.argtypes = [P] * 12
    lib.orc_tree_export.restype = None
    lib.orc_walk.argtypes = [P, P, i64, d, P, d, ctypes.c_int, P, P, P, P, P, P, P, i64]
    lib.orc_walk.restype = ctypes.c_int
    lib.orc_tree_quad.argtypes = [P, P]
    lib.orc_tree_quad.restype = None
    lib.orc_cell_term.argtypes = [P, P, d, P, d, ctypes.c_int, P, P]
    lib.orc_cell_term.restype = None
    lib.orc_sph_kernel.argtypes = [d, d]
    lib.orc_sph_kernel.restype = d
    lib.orc_neighbours.argtypes = [P, P, i64, d, P, P, P, i64, P]
    lib.orc_neighbours.restype = ctypes.c_int
    lib.orc_neighbours_brute.argtypes = [P, P, i64, P, i64, d, P, P]
    lib.orc_neighbours_brute.restype = ctypes.c_int
    lib.orc_leapfrog.argtypes = [P, P, P, i64, d, d, i64, P, P]
    lib.orc_leapfrog.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _as_pos(pos):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    if pos.ndim != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be [n, 3]")
    return pos


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    _load().orc_set_num_threads(int(n))


def direct(pos, mass, eps, targets=None):
    """Direct sum of Eq. (1) for ``targets`` (all particles if None).

    Returns ``(acc [nt,3], pot [nt], amag [nt])`` in float64, where ``amag`` is
    the sum of the magnitudes of the acceleration terms.
    """
    lib = _load()
    pos = _as_pos(pos)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    amag = np.zeros(nt)
    rc = lib.orc_direct(_ptr(pos), _ptr(mass), n, _ptr(tg), nt, float(eps),
                        _ptr(acc), _ptr(pot), _ptr(amag))
    if rc != 0:
        raise ValueError("orc_direct rejected its arguments")
    return acc, pot, amag


class Tree:
    """Oracle oct-tree of ``n`` particles (Sec. 4.1), nodes in depth-first preorder."""

    def __init__(self, pos, mass):
        lib = _load()
        self.pos = _as_pos(pos)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        if self.mass.shape != (self.pos.shape[0],):
            raise ValueError("mass must be [n]")
        self.n = self.pos.shape[0]
        self._h = lib.orc_tree_build(_ptr(self.pos), _ptr(self.mass), self.n)
        if not self._h:
            raise MemoryError("oracle tree build failed")
        self.n_nodes = int(lib.orc_tree_nodes(self._h))
        lo = np.zeros(3)
        L = np.zeros(1)
        lib.orc_tree_cube(self._h, _ptr(lo), _ptr(L))
        self.lo, self.L = lo, float(L[0])
        m = self.n_nodes
        self.level = np.zeros(m, np.int32)
        self.first = np.zeros(m, np.int32)
        self.count = np.zeros(m, np.int32)
        self.next = np.zeros(m, np.int32)
        self.leaf = np.zeros(m, np.int8)
        self.cell = np.zeros((m, 3), np.int64)
        self.com = np.zeros((m, 3))
        self.M = np.zeros(m)
        self.s = np.zeros(m)
        self.l = np.zeros(m)
        self.perm = np.zeros(self.n, np.int64)
        lib.orc_tree_export(self._h, _ptr(self.level), _ptr(self.first), _ptr(self.count),
                            _ptr(self.next), _ptr(self.leaf), _ptr(self.cell), _ptr(self.com),
                            _ptr(self.M), _ptr(self.s), _ptr(self.l), _ptr(self.perm))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().orc_tree_free(h)
            self._h = None

    @property
    def B(self):
        """Second moments [n_nodes, 6] (xx xy xz yy yz zz) of every node about its centre of mass."""
        out = np.zeros((self.n_nodes, 6))
        _load().orc_tree_quad(self._h, _ptr(out))
        return out

    def walk(self, theta, eps, targets=None, theta_per_target=None, maxlen=0, order=1):
        """Fig. 3 walk for ``targets`` (original indices; all if None).

        ``order`` 1: monopole cell terms (Eq. (1) with the cell's mass at its centre of
        mass); 2: the second-order expansion of the softened cell potential (quadrupole).

        Returns a dict with ``acc [nt,3]``, ``pot``, ``amag``, ``n_pp``, ``n_pc``,
        ``hash`` (uint64 ordered-list hash) and, if ``maxlen`` > 0, ``lists``
        ([nt, maxlen] int64 words, -1 padded; word = j<<1 for a particle term with
        original index j, node<<1|1 for a cell term with preorder id node).
        """
        lib = _load()
        tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
        nt = self.n if tg is None else tg.shape[0]
        tpt = None
        if theta_per_target is not None:
            tpt = np.ascontiguousarray(theta_per_target, dtype=np.float64)
            if tpt.shape != (nt,):
                raise ValueError("theta_per_target must have one value per target")
        out = dict(acc=np.zeros((nt, 3)), pot=np.zeros(nt), amag=np.zeros(nt),
                   n_pp=np.zeros(nt, np.int64), n_pc=np.zeros(nt, np.int64),
                   hash=np.zeros(nt, np.uint64))
        lists = None
        if maxlen > 0:
            lists = np.full((nt, maxlen), -1, np.int64)
        rc = lib.orc_walk(self._h, _ptr(tg), nt, float(theta), _ptr(tpt), float(eps), int(order),
                          _ptr(out["acc"]), _ptr(out["pot"]), _ptr(out["amag"]),
                          _ptr(out["n_pp"]), _ptr(out["n_pc"]), _ptr(out["hash"]),
                          _ptr(lists), int(maxlen))
        if rc != 0:
            raise ValueError("orc_walk rejected its arguments")
        if lists is not None:
            out["lists"] = lists
        return out


def leapfrog(pos, vel, mass, eps, dt, steps, acc=None):
    """Kick-drift-kick leapfrog on the direct-sum forces (Sec. 1: force, integrate, repeat).

    Returns (pos, vel, acc, pot) after ``steps`` steps of size ``dt`` (copies; the inputs are not
    changed).  ``acc`` is a(x) of the initial positions (computed if None)."""
    lib = _load()
    pos = np.array(_as_pos(pos), dtype=np.float64)
    vel = np.array(_as_pos(vel), dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if acc is None:
        acc, pot, _ = direct(pos, mass, eps)
    acc = np.array(acc, dtype=np.float64)
    pot = np.zeros(n)
    if lib.orc_leapfrog(_ptr(pos), _ptr(vel), _ptr(mass), n, float(eps), float(dt), int(steps), _ptr(acc),
                        _ptr(pot)) != 0:
        raise ValueError("orc_leapfrog rejected its arguments")
    return pos, vel, acc, pot


def sph_kernel(r, h):
    """M4 cubic spline W(r, h) of compact support 2h (three dimensions)."""
    return float(_load().orc_sph_kernel(float(r), float(h)))


def neighbours_brute(pos, mass, radius, targets=None):
    """Brute force over all pairs: (count [nt], rho [nt]) of the neighbours within ``radius``."""
    lib = _load()
    pos = _as_pos(pos)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = pos.shape[0] if tg is None else tg.shape[0]
    cnt = np.zeros(nt, np.int64)
    rho = np.zeros(nt)
    if lib.orc_neighbours_brute(_ptr(pos), _ptr(mass), pos.shape[0], _ptr(tg), nt, float(radius), _ptr(cnt),
                                _ptr(rho)) != 0:
        raise ValueError("orc_neighbours_brute rejected its arguments")
    return cnt, rho


def cell_term(xi, com, M, B, eps, order=2):
    """One particle-cell term at target xi of a cell with mass M, centre of mass com and second
    moments B (xx xy xz yy yz zz); returns (acc [3], pot)."""
    xi = np.ascontiguousarray(xi, np.float64)
    com = np.ascontiguousarray(com, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    acc = np.zeros(3)
    pot = np.zeros(1)
    _load().orc_cell_term(_ptr(xi), _ptr(com), float(M), _ptr(B), float(eps), int(order), _ptr(acc), _ptr(pot))
    return acc, float(pot[0])


def _tree_neighbours(self, radius, targets=None, maxlen=0):
    """General tree walk of Fig. 4 as a neighbour search: per target the count of particles within
    ``radius``, their ordered hash (walk order), optional lists and the SPH density."""
    lib = _load()
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = self.n if tg is None else tg.shape[0]
    out = dict(count=np.zeros(nt, np.int64), hash=np.zeros(nt, np.uint64), rho=np.zeros(nt))
    lists = np.full((nt, maxlen), -1, np.int64) if maxlen > 0 else None
    if lib.orc_neighbours(self._h, _ptr(tg), nt, float(radius), _ptr(out["count"]), _ptr(out["hash"]),
                          _ptr(lists), int(maxlen), _ptr(out["rho"])) != 0:
        raise ValueError("orc_neighbours rejected its arguments")
    if lists is not None:
        out["lists"] = lists
    return out


Tree.neighbours = _tree_neighbours


def rms_rel_err(a, a_ref):
    """RMS over particles of |a - a_ref| / |a_ref| (the RMS form of Eq. (4))."""
    a = np.asarray(a, np.float64)
    a_ref = np.asarray(a_ref, np.float64)
    if a.ndim == 1:
        r = np.abs(a - a_ref) / np.abs(a_ref)
    else:
        r = np.linalg.norm(a - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
    return float(np.sqrt(np.mean(r * r)))


def mean_rel_err(a, a_ref):
    """Mean over particles of |a - a_ref| / |a_ref|, Eq. (4)."""
    a = np.asarray(a, np.float64)
    a_ref = np.asarray(a_ref, np.float64)
    if a.ndim == 1:
        r = np.abs(a - a_ref) / np.abs(a_ref)
    else:
        r = np.linalg.norm(a - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
    return float(np.mean(r))
