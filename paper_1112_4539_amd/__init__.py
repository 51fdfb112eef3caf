"""gfx950 Barnes-Hut tree forces (arXiv:1112.4539), Python binding of ``libbh.so``.

Argument marshalling only: every step of the method runs in the library's HIP
kernels (declared in ``include/bh.h``).  torch provides device memory and the
stream; it must be imported before the library is loaded so that both use
the same HIP runtime.  There is no fallback: if ``libbh.so`` is missing or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

__all__ = ["Tree", "Forest", "Graph", "build_tree", "build_forest", "direct", "forces_noalloc", "leapfrog_step", "workspace_bytes",
           "forest_workspace_bytes", "load", "THETA_MAX", "BHError", "FP32", "FP64", "WalkConfig"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbh.so")
FP32, FP64 = 0, 1
THETA_MAX = 2.0 / math.sqrt(3.0)

_lib = None


class BHError(RuntimeError):
    pass


class WalkConfig(ctypes.Structure):
    """``bh_walk_config``: a launch shape of the walk and its measured time."""
    _fields_ = [("waves_per_block", ctypes.c_int), ("xcd_chunk", ctypes.c_int), ("lds_share", ctypes.c_int),
                ("persistent", ctypes.c_int), ("targets_per_lane", ctypes.c_int), ("ms", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def load():
    """Load ``libbh.so`` (built by ``paper_1112_4539_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BHError(f"{LIB_PATH} is not built; run `python paper_1112_4539_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "bh_last_error": ([], ctypes.c_char_p),
        "bh_version": ([], i32),
        "bh_workspace_bytes": ([i64, i32], i64),
        "bh_forest_workspace_bytes": ([i64, i64, i32], i64),
        "bh_build_tree": ([P, P, i64, i32, P, i64, P, P], i32),
        "bh_build_forest": ([P, P, P, i64, i64, i32, P, i64, P, P], i32),
        "bh_forest_roots": ([P, P, P], i32),
        "bh_graph_create": ([P, d, d, P, P, P, P], i32),
        "bh_graph_launch": ([P, P], i32),
        "bh_graph_release": ([P], None),
        "bh_autotune": ([P, d, d, P, P, i32, P, P, P, i32, P], i32),
        "bh_tree_check": ([P, P], i32),
        "bh_tree_stats": ([P, P, P, P, P], i32),
        "bh_forces": ([P, d, d, P, P, P], i32),
        "bh_forces_theta": ([P, P, d, P, P, P], i32),
        "bh_forces_noalloc": ([P, P, i64, i32, d, d, P, P, P], i32),
        "bh_walk_stats": ([P, d, P, d, P, P, P, P, P, i64, P, P], i32),
        "bh_tree_export": ([P, P, P, P], i32),
        "bh_set_walk_config": ([P, i32, i32, i32, i32, i32, i32], i32),
        "bh_set_timing": ([P, i32], i32),
        "bh_set_expansion_order": ([P, i32], i32),
        "bh_tree_moments2": ([P, P, P], i32),
        "bh_neighbours": ([P, d, P, P, P, i64, P, P], i32),
        "bh_walk_order": ([P, P, P], i32),
        "bh_leapfrog_step": ([P, P, P, P, P, P, i64, i32, d, d, d, i32, i32, P, i64, P], i32),
        "bh_walk_time_ms": ([P, P], i32),
        "bh_tree_release": ([P], None),
        "bh_direct": ([P, P, i64, i32, P, i64, d, P, P, P], i32),
        "bh_features": ([P, P, P], i32),
        "bh_group_error": ([P, P, P, d, d, P, P, P], i32),
        "bh_mlp_sizes": ([i64, P, P, P, P], i32),
        "bh_mlp_prepare": ([P, P, P], i32),
        "bh_mlp_infer": ([P, P, P, P, i64, ctypes.c_float, ctypes.c_float, P, P], i32),
        "bh_mlp_grad": ([P, P, P, P, P, P, i64, P, P, P], i32),
        "bh_mlp_adam": ([P, P, P, P, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P],
                        i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        msg = load().bh_last_error().decode()
        if rc == -1:
            raise ValueError(msg)
        raise BHError(f"status {rc}: {msg}")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _prec_of(dtype):
    if dtype == torch.float32:
        return FP32
    if dtype == torch.float64:
        return FP64
    raise TypeError("positions and masses must be float32 or float64")


def workspace_bytes(n, prec):
    v = load().bh_workspace_bytes(int(n), int(prec))
    if v < 0:
        raise ValueError(f"invalid n={n} or precision={prec}")
    return int(v)


def forest_workspace_bytes(n, n_clusters, prec):
    v = load().bh_forest_workspace_bytes(int(n), int(n_clusters), int(prec))
    if v < 0:
        raise ValueError(f"invalid n={n}, n_clusters={n_clusters} or precision={prec}")
    return int(v)


NODE_DTYPE = None


def _node_dtype():
    import numpy as np
    global NODE_DTYPE
    if NODE_DTYPE is None:
        NODE_DTYPE = np.dtype([("com", "<f8", (3,)), ("M", "<f8"), ("l", "<f8"), ("s", "<f8"),
                               ("next", "<i4"), ("first", "<i4"), ("count", "<i4"), ("meta", "<i4")])
    return NODE_DTYPE


class Tree:
    """Oct-tree of one particle set on the GPU (``bh_build_tree``).

    ``pos`` [n,3] and ``mass`` [n] are CUDA tensors of one float dtype; the tree
    keeps references to them and to its workspace tensor.
    """

    def __init__(self, pos, mass, workspace=None, offsets=None):
        lib = load()
        if pos.device.type != "cuda" or mass.device.type != "cuda":
            raise ValueError("pos and mass must be device tensors")
        if pos.dtype != mass.dtype:
            raise TypeError("pos and mass must have the same dtype")
        self.prec = _prec_of(pos.dtype)
        self.pos = pos.contiguous()
        self.mass = mass.contiguous()
        if self.pos.dim() != 2 or self.pos.shape[1] != 3 or self.mass.shape != (self.pos.shape[0],):
            raise ValueError("pos must be [n,3] and mass [n]")
        self.n = int(self.pos.shape[0])
        self.device = self.pos.device
        self.offsets = None
        self.n_clusters = 1
        self.order = 1
        if offsets is not None:
            if offsets.dtype != torch.int64 or offsets.device != self.device or offsets.dim() != 1 \
                    or offsets.shape[0] < 2:
                raise ValueError("offsets must be an int64 device tensor [n_clusters+1]")
            self.offsets = offsets.contiguous()
            self.n_clusters = int(offsets.shape[0]) - 1
        need = forest_workspace_bytes(self.n, self.n_clusters, self.prec)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        h = ctypes.c_void_p()
        _check(lib.bh_build_forest(_ptr(self.pos), _ptr(self.mass), _ptr(self.offsets), self.n_clusters, self.n,
                                   self.prec, _ptr(workspace), workspace.numel(), _stream(self.device),
                                   ctypes.byref(h)))
        self._h = h
        self._release = lib.bh_tree_release  # kept for __del__ during interpreter shutdown

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._release(h)
            self._h = None

    @property
    def dtype(self):
        return self.pos.dtype

    def check(self):
        """Synchronise; raise ValueError if an input coordinate or mass was not finite."""
        _check(load().bh_tree_check(self._h, _stream(self.device)))

    def stats(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().bh_tree_stats(self._h, _stream(self.device), ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
        return dict(n_nodes=a.value, n_leaves=b.value, n_internal=c.value)

    def set_walk_config(self, waves_per_block=1, xcd_chunk=-1, target_order=2, lds_share=0, persistent=0,
                        targets_per_lane=1):
        _check(load().bh_set_walk_config(self._h, int(waves_per_block), int(xcd_chunk), int(target_order),
                                         int(lds_share), int(persistent), int(targets_per_lane)))

    def autotune(self, theta, eps, acc=None, pot=None, reps=2, max_tried=64):
        """Pick the walk shape by measurement (``bh_autotune``); returns (best, tried) as dicts."""
        acc, pot = self._outs(acc, pot)
        best = WalkConfig()
        tried = (WalkConfig * max_tried)()
        nt = ctypes.c_int()
        _check(load().bh_autotune(self._h, float(theta), float(eps), _ptr(acc), _ptr(pot), int(reps),
                                  _stream(self.device), ctypes.byref(best), tried, int(max_tried),
                                  ctypes.byref(nt)))
        return best.as_dict(), [tried[i].as_dict() for i in range(min(nt.value, max_tried))]

    def roots(self):
        """Preorder id of every cluster's root, plus the node count (``bh_forest_roots``)."""
        r = torch.empty((self.n_clusters + 1,), dtype=torch.int32, device=self.device)
        _check(load().bh_forest_roots(self._h, _ptr(r), _stream(self.device)))
        return r

    @property
    def n_groups(self):
        return (self.n + 63) // 64

    def features(self):
        """Features [ceil(n/64), 8] float32 of the walk groups (``bh_features``)."""
        X = torch.empty((self.n_groups, 8), dtype=torch.float32, device=self.device)
        _check(load().bh_features(self._h, _ptr(X), _stream(self.device)))
        return X

    def group_error(self, acc, acc_ref, theta=0.0, target=0.0, label=None):
        """Per-group RMS relative force error against acc_ref (float64); optionally raises
        label[g] to theta where it is within target (``bh_group_error``)."""
        acc, _ = self._outs(acc, None)
        if acc_ref.dtype != torch.float64 or acc_ref.shape != (self.n, 3) or not acc_ref.is_contiguous():
            raise ValueError("acc_ref must be a contiguous float64 [n,3] device tensor")
        rms = torch.empty((self.n_groups,), dtype=torch.float64, device=self.device)
        if label is not None and (label.dtype != torch.float32 or label.shape != (self.n_groups,)):
            raise ValueError("label must be float32 [n_groups]")
        _check(load().bh_group_error(self._h, _ptr(acc), _ptr(acc_ref), float(theta), float(target), _ptr(rms),
                                     _ptr(label), _stream(self.device)))
        return rms

    def graph(self, theta, eps, acc, pot):
        """Capture build + forces into acc/pot as one HIP graph (``bh_graph_create``)."""
        return Graph(self, theta, eps, acc, pot)

    def neighbours(self, radius, maxlen=0, density=True):
        """Neighbour search within ``radius`` (``bh_neighbours``): dict of count [n] int32, hash [n],
        optional lists [n, maxlen] (caller indices, walk order) and the SPH density rho [n]."""
        count = torch.empty((self.n,), dtype=torch.int32, device=self.device)
        hsh = torch.empty((self.n,), dtype=torch.int64, device=self.device)
        lists = torch.full((self.n, maxlen), -1, dtype=torch.int64, device=self.device) if maxlen > 0 else None
        rho = torch.empty((self.n,), dtype=self.dtype, device=self.device) if density else None
        _check(load().bh_neighbours(self._h, float(radius), _ptr(count), _ptr(hsh), _ptr(lists), int(maxlen),
                                    _ptr(rho), _stream(self.device)))
        out = dict(count=count, hash=hsh)
        if lists is not None:
            out["lists"] = lists
        if rho is not None:
            out["rho"] = rho
        return out

    def walk_order(self):
        """Caller indices of the targets in the order the walk takes them (``bh_walk_order``)."""
        out = torch.empty((max(self.n, 1),), dtype=torch.int32, device=self.device)
        _check(load().bh_walk_order(self._h, _ptr(out), _stream(self.device)))
        return out[: self.n]

    def moments2(self):
        """Second moments [n_nodes, 6] float64 (xx xy xz yy yz zz) of every node about its centre
        of mass (``bh_tree_moments2``)."""
        m = self.stats()["n_nodes"]
        B = torch.empty((max(m, 1), 6), dtype=torch.float64, device=self.device)
        _check(load().bh_tree_moments2(self._h, _ptr(B), _stream(self.device)))
        return B[:m]

    def set_order(self, order):
        """Particle-cell terms of later walks: 1 monopole (Eq. (1)), 2 with the quadrupole
        correction (``bh_set_expansion_order``)."""
        _check(load().bh_set_expansion_order(self._h, int(order)))
        self.order = int(order)

    def set_timing(self, enable=True):
        _check(load().bh_set_timing(self._h, 1 if enable else 0))

    def walk_time_ms(self):
        ms = ctypes.c_float()
        _check(load().bh_walk_time_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)

    def _outs(self, acc, pot):
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=self.dtype, device=self.device)
        if pot is None:
            pot = torch.empty((self.n,), dtype=self.dtype, device=self.device)
        if acc.dtype != self.dtype or pot.dtype != self.dtype or not acc.is_contiguous() \
                or not pot.is_contiguous() or acc.shape != (self.n, 3) or pot.shape != (self.n,):
            raise ValueError("acc must be [n,3] and pot [n], contiguous, in the tree's dtype")
        return acc, pot

    def _theta_group(self, theta_group):
        if theta_group is None:
            return None
        g = (self.n + 63) // 64
        if theta_group.shape != (g,) or theta_group.dtype != torch.float32 or theta_group.device != self.device:
            raise ValueError(f"theta_group must be a float32 device tensor of shape [{g}]")
        return theta_group.contiguous()

    def forces(self, theta=0.5, eps=0.0, acc=None, pot=None, theta_group=None):
        """Tree-walk accelerations [n,3] and potentials [n] (``bh_forces`` / ``bh_forces_theta``)."""
        acc, pot = self._outs(acc, pot)
        lib = load()
        tg = self._theta_group(theta_group)
        if tg is None:
            _check(lib.bh_forces(self._h, float(theta), float(eps), _ptr(acc), _ptr(pot), _stream(self.device)))
        else:
            _check(lib.bh_forces_theta(self._h, _ptr(tg), float(eps), _ptr(acc), _ptr(pot),
                                       _stream(self.device)))
        return acc, pot

    def walk_stats(self, theta=0.5, eps=0.0, theta_group=None, maxlen=0):
        """Forces plus per-particle (particle terms, cell terms), list hash, nodes visited per
        64-target group, and an optional list dump."""
        acc, pot = self._outs(None, None)
        counts = torch.empty((self.n, 2), dtype=torch.int32, device=self.device)
        hsh = torch.empty((self.n,), dtype=torch.int64, device=self.device)
        steps = torch.zeros(((self.n + 63) // 64,), dtype=torch.int32, device=self.device)
        lists = None
        if maxlen > 0:
            lists = torch.full((self.n, maxlen), -1, dtype=torch.int64, device=self.device)
        tg = self._theta_group(theta_group)
        _check(load().bh_walk_stats(self._h, float(theta), _ptr(tg), float(eps), _ptr(acc), _ptr(pot),
                                    _ptr(counts), _ptr(hsh), _ptr(lists), int(maxlen), _ptr(steps),
                                    _stream(self.device)))
        out = dict(acc=acc, pot=pot, counts=counts, hash=hsh, group_steps=steps)
        if lists is not None:
            out["lists"] = lists
        return out

    def export(self):
        """Node records (numpy structured array, preorder) and perm (Morton position -> caller index)."""
        import numpy as np
        st = self.stats()
        m = st["n_nodes"]
        nodes = torch.empty((max(m, 1) * 64,), dtype=torch.uint8, device=self.device)
        perm = torch.empty((max(self.n, 1),), dtype=torch.int32, device=self.device)
        _check(load().bh_tree_export(self._h, _ptr(nodes), _ptr(perm), _stream(self.device)))
        rec = nodes.cpu().numpy()[: m * 64].view(_node_dtype())
        return rec, perm.cpu().numpy()[: self.n].astype(np.int64)


class Graph:
    """The captured pipeline of a tree: every launch rebuilds from the tree's input tensors
    (their current contents) and writes the forces to the captured acc/pot."""

    def __init__(self, tree, theta, eps, acc, pot):
        acc, pot = tree._outs(acc, pot)
        self.tree, self.acc, self.pot = tree, acc, pot
        g = ctypes.c_void_p()
        _check(load().bh_graph_create(tree._h, float(theta), float(eps), _ptr(acc), _ptr(pot),
                                      _stream(tree.device), ctypes.byref(g)))
        self._g = g
        self._release = load().bh_graph_release

    def launch(self):
        _check(load().bh_graph_launch(self._g, _stream(self.tree.device)))
        return self.acc, self.pot

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value:
            self._release(g)
            self._g = None


Forest = Tree


class MLP:
    """Parameters and kernels of the opening-parameter network (``bh_mlp_*``).

    ``params`` FP32 [4801] (W1, b1, W2, b2, w3, b3), ``norm`` FP32 [16] (mu, 1/sd), bf16
    weight copies kept in step by ``prepare`` / ``adam``.
    """

    def __init__(self, params, norm, device="cuda"):
        lib = load()
        npar, ngrad, nwb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.bh_mlp_sizes(1, ctypes.byref(npar), ctypes.byref(ngrad), ctypes.byref(nwb), None))
        self.n_param, self.n_grad = npar.value, ngrad.value
        self.device = torch.device(device)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        self.norm = torch.as_tensor(norm, dtype=torch.float32).to(self.device).contiguous()
        if self.params.shape != (self.n_param,) or self.norm.shape != (16,):
            raise ValueError(f"params must be [{self.n_param}] and norm [16]")
        self.wbf16 = torch.zeros((nwb.value,), dtype=torch.int16, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.prepare()

    def prepare(self):
        _check(load().bh_mlp_prepare(_ptr(self.params), _ptr(self.wbf16), _stream(self.device)))

    def infer(self, X, alpha=1.0, fallback=0.5):
        X = X.contiguous()
        theta = torch.empty((X.shape[0],), dtype=torch.float32, device=self.device)
        _check(load().bh_mlp_infer(_ptr(self.params), _ptr(self.wbf16), _ptr(self.norm), _ptr(X), X.shape[0],
                                   float(alpha), float(fallback), _ptr(theta), _stream(self.device)))
        return theta

    def grad(self, X, target, rows_idx):
        """Gradient of mean((sigmoid(z) - target)^2) over rows_idx; the last entry is the loss."""
        lib = load()
        part = ctypes.c_int64()
        B = int(rows_idx.shape[0])
        _check(lib.bh_mlp_sizes(B, None, None, None, ctypes.byref(part)))
        partial = torch.empty((part.value,), dtype=torch.float32, device=self.device)
        g = torch.empty((self.n_grad,), dtype=torch.float32, device=self.device)
        _check(lib.bh_mlp_grad(_ptr(self.params), _ptr(self.wbf16), _ptr(self.norm), _ptr(X.contiguous()),
                               _ptr(target.contiguous()), _ptr(rows_idx.to(torch.int32).contiguous()), B,
                               _ptr(partial), _ptr(g), _stream(self.device)))
        return g

    def adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(load().bh_mlp_adam(_ptr(self.params), _ptr(grad), _ptr(self.m), _ptr(self.v), self.step, float(lr),
                                  float(beta1), float(beta2), float(eps), _ptr(self.wbf16), _stream(self.device)))


def build_tree(pos, mass, workspace=None):
    return Tree(pos, mass, workspace)


def build_forest(pos, mass, offsets, workspace=None):
    """One tree per cluster [offsets[k], offsets[k+1]) in one build (``bh_build_forest``)."""
    return Tree(pos, mass, workspace, offsets=offsets)


def leapfrog_step(pos, vel, mass, acc, pot, dt, theta, eps, order=1, reorder=False, ids=None, workspace=None):
    """One kick-drift-kick step of the time loop (``bh_leapfrog_step``), in place on the caller's
    device state; ``acc`` must hold the forces of the current positions.  With ``reorder`` the
    state (and ``ids``) is permuted into the new tree's Morton order."""
    lib = load()
    prec = _prec_of(pos.dtype)
    n = int(pos.shape[0])
    for t, shape in ((pos, (n, 3)), (vel, (n, 3)), (acc, (n, 3)), (mass, (n,)), (pot, (n,))):
        if t.dtype != pos.dtype or tuple(t.shape) != shape or not t.is_contiguous() or t.device != pos.device:
            raise ValueError("pos/vel/acc must be [n,3] and mass/pot [n], contiguous, one dtype and device")
    if ids is not None and (ids.dtype != torch.int64 or ids.shape != (n,) or not ids.is_contiguous()):
        raise ValueError("ids must be a contiguous int64 [n] tensor")
    need = workspace_bytes(n, prec)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=pos.device)
    _check(lib.bh_leapfrog_step(_ptr(pos), _ptr(vel), _ptr(mass), _ptr(acc), _ptr(pot), _ptr(ids), n, prec,
                                float(dt), float(theta), float(eps), int(order), 1 if reorder else 0,
                                _ptr(workspace), workspace.numel(), _stream(pos.device)))
    return workspace


NOALLOC_MAX_N = 65536


def forces_noalloc(pos, mass, theta, eps, acc, pot):
    """Build + forces with the library's static scratch array (``bh_forces_noalloc``): no device
    memory is allocated, by the library or here; acc [n,3] and pot [n] are the caller's."""
    lib = load()
    prec = _prec_of(pos.dtype)
    n = int(pos.shape[0])
    for t, shape in ((pos, (n, 3)), (mass, (n,)), (acc, (n, 3)), (pot, (n,))):
        if t.dtype != pos.dtype or tuple(t.shape) != shape or not t.is_contiguous() or t.device != pos.device:
            raise ValueError("pos/acc must be [n,3] and mass/pot [n], contiguous, one dtype and device")
    with torch.cuda.device(pos.device):
        _check(lib.bh_forces_noalloc(_ptr(pos), _ptr(mass), n, prec, float(theta), float(eps), _ptr(acc),
                                     _ptr(pot), _stream(pos.device)))
    return acc, pot


def direct(pos, mass, eps, targets=None):
    """Brute-force Eq. (1) for ``targets`` (int64 device tensor of caller indices; all if None)."""
    lib = load()
    prec = _prec_of(pos.dtype)
    pos = pos.contiguous()
    mass = mass.contiguous()
    n = int(pos.shape[0])
    if targets is None:
        targets = torch.arange(n, dtype=torch.int64, device=pos.device)
    targets = targets.to(torch.int64).contiguous()
    nt = int(targets.shape[0])
    acc = torch.empty((nt, 3), dtype=pos.dtype, device=pos.device)
    pot = torch.empty((nt,), dtype=pos.dtype, device=pos.device)
    _check(lib.bh_direct(_ptr(pos), _ptr(mass), n, prec, _ptr(targets), nt, float(eps), _ptr(acc), _ptr(pot),
                         _stream(pos.device)))
    return acc, pot
