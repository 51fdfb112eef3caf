"""Learned opening parameter: labelling, training and use of the theta network.

Host orchestration: the physics and the network run in the library's kernels
(features, direct sum, force walks, per-group errors, the MLP's forward,
gradient and Adam passes); this module chooses what to run.  Host arithmetic
is limited to the label allocation below (an argmin over the theta grid with
a bisected multiplier), the feature normalisation constants (eight means and
standard deviations of the training features) and the minibatch shuffles.

Groups: a theta belongs to a walk group, the 64 targets a wavefront walks
together (runs of 64 of the tree's target order, by default the Hilbert
order), so that one wavefront walks with one theta.

Labels: a training snapshot is walked at every theta of the grid 0.20, 0.25,
..., 1.00; for every walk group g this gives its RMS relative force error
R[k, g] against the FP64 direct sum and its cost C[k, g] (nodes its wavefront
visits).  The label is the cost-optimal allocation for the snapshot:
theta*_g = grid[argmin_k C[k, g] + lambda n_g R[k, g]^2], with the multiplier
lambda bisected so that the snapshot's overall RMS error is the target (1e-3)
-- the least total cost at that error that per-group choices on the grid can
reach.  (Labelling each group with the largest theta that keeps its own error
within the target spends interactions where they buy little accuracy.)  The
allocation can also be taken over a random sample of the groups of a large
particle set (label_sampled): the direct sum then runs for the sampled groups'
targets only, which makes labels affordable at the resolution the network is
used at.  The network is fitted to t = (theta* - 0.2) / 0.8 with the loss
mean((sigmoid(z) - t)^2).  At use, theta_g = min(alpha * theta(x_g),
1.15), with alpha a single scale that the caller sets (e.g. by bisection to a
global error target); a non-finite output falls back to a fixed theta.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

import paper_1112_4539_amd as bh
from paper_1112_4539_amd import inputs, metrics

THETA_GRID = tuple(round(0.20 + 0.05 * k, 2) for k in range(17))
TARGET = 1e-3
N_PARAM = 4801
WEIGHTS_FORMAT = "theta-mlp-8-64-64-1"
# the network shipped with the package (written by train_theta.py)
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "theta_clumpy4m.json")


def init_params(seed):
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases, in the flat layout W1, b1, W2, b2, w3, b3."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.uniform(-1, 1, 512) / math.sqrt(8), np.zeros(64),
                           rng.uniform(-1, 1, 4096) / math.sqrt(64), np.zeros(64),
                           rng.uniform(-1, 1, 64) / math.sqrt(64), np.zeros(1)]).astype(np.float32)


def _dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def allocate(R, C, n_g, target):
    """Cost-optimal grid index per group: argmin_k C[k,g] + lam n_g R[k,g]^2 with lam such that
    sqrt(sum_g n_g R[k_g,g]^2 / N) is at most (and close to) the target.

    Entries whose error or cost is not finite are never chosen; a group with no finite entry at
    all takes grid index 0 (the smallest theta) and is left out of the error sum, so that one
    bad group cannot move the allocation of the others."""
    R = np.asarray(R, np.float64)
    C = np.asarray(C, np.float64)
    n_g = np.asarray(n_g, np.float64)
    E = n_g[None, :] * R * R
    ok = np.isfinite(E) & np.isfinite(C)
    E = np.where(ok, E, np.inf)
    Cm = np.where(ok, C, np.inf)
    dead = ~ok.any(axis=0)
    live = ~dead
    N = float(n_g[live].sum()) if live.any() else 1.0
    cols = np.arange(R.shape[1])

    def pick(lam):
        with np.errstate(invalid="ignore"):
            k = np.argmin(Cm + lam * E, axis=0)
        k[dead] = 0
        return k, np.sqrt(E[k[live], cols[live]].sum() / N)

    lo, hi = 0.0, 40.0      # log10 of lambda
    k, err = pick(10.0 ** hi)
    if err > target:
        return k
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        km, em = pick(10.0 ** mid)
        if em <= target:
            hi, k = mid, km
        else:
            lo = mid
    return k


def label_snapshot(pos, mass, eps, grid=THETA_GRID, target=TARGET):
    """Features [G, 8] and labels [G] (device float32) of one particle set (FP32 walk), plus the
    per-group error and cost tables R, C [len(grid), G]."""
    gp, gm = _dev(pos, torch.float32), _dev(mass, torch.float32)
    T = bh.Tree(gp, gm)
    X = T.features()
    # the reference sees exactly the FP32 values the walk sees
    a_ref, _ = bh.direct(gp.double(), gm.double(), eps)
    R, C = [], []
    for th in grid:
        st = T.walk_stats(th, eps)
        R.append(T.group_error(st["acc"], a_ref))
        C.append(st["group_steps"].double())
    R = torch.stack(R).cpu().numpy()
    C = torch.stack(C).cpu().numpy()
    n_g = np.full(T.n_groups, 64.0)
    n_g[-1] = T.n - 64 * (T.n_groups - 1)
    k = allocate(R, C, n_g, target)
    label = torch.tensor(np.asarray(grid, np.float32)[k], device="cuda")
    return X, label, R, C


def label_sampled(pos, mass, eps, n_groups, seed, grid=THETA_GRID, target=TARGET):
    """Features [S, 8] and labels [S] (device float32) of S = n_groups walk groups sampled
    (without replacement, from default_rng(seed); the last, possibly ragged group excluded) from one
    particle set, plus their error and cost tables R, C [len(grid), S].  Labels as in
    label_snapshot, the allocation taken over the sample: for large sets the direct sum then covers
    only the sampled groups' 64 S targets."""
    gp, gm = _dev(pos, torch.float32), _dev(mass, torch.float32)
    T = bh.Tree(gp, gm)
    X = T.features()
    n, G = T.n, T.n_groups
    n_groups = min(n_groups, G - 1)
    gs = np.sort(np.random.default_rng(seed).choice(G - 1, n_groups, replace=False))
    order = T.walk_order().cpu().numpy().astype(np.int64)  # caller indices in walk order
    targets = order[(gs[:, None] * 64 + np.arange(64)[None, :]).ravel()]
    tg = torch.tensor(targets, device="cuda")
    a_s, _ = bh.direct(gp.double(), gm.double(), eps, tg)
    a_ref = torch.zeros((n, 3), dtype=torch.float64, device="cuda")  # groups outside the sample: unused
    a_ref[tg] = a_s
    gsel = torch.tensor(gs, device="cuda")
    R, C = [], []
    for th in grid:
        st = T.walk_stats(th, eps)
        R.append(T.group_error(st["acc"], a_ref)[gsel])
        C.append(st["group_steps"].double()[gsel])
    R = torch.stack(R).cpu().numpy()
    C = torch.stack(C).cpu().numpy()
    k = allocate(R, C, np.full(n_groups, 64.0), target)
    label = torch.tensor(np.asarray(grid, np.float32)[k], device="cuda")
    return X[gsel].contiguous(), label, R, C


def build_dataset_sampled(seeds, n, n_groups, log=None):
    """Training rows from clumpy fields of n particles (one per seed, eps 1e-4), n_groups sampled
    groups each: labels at the resolution the network is to be used at."""
    Xs, Ls = [], []
    for s in seeds:
        pos, mass = inputs.clumpy(n, s)
        X, lab, _, _ = label_sampled(pos, mass, 1e-4, n_groups, s)
        Xs.append(X)
        Ls.append(lab)
        if log:
            log(f"[learn] snapshot seed={s} n={n} sampled groups={len(lab)} mean label={float(lab.mean()):.3f}")
    return torch.cat(Xs), torch.cat(Ls)


def training_snapshot(seed, n=262_144):
    """Training set member: even seeds a Plummer sphere (eps 0.005), odd seeds the clumpy field
    recipe (25% uniform + 64 clumps, eps 1e-4)."""
    if seed % 2 == 0:
        pos, mass = inputs.plummer(n, seed)
        return pos, mass, 0.005
    pos, mass = inputs.clumpy(n, seed)
    return pos, mass, 1e-4


def build_dataset(seeds, n=262_144, log=None):
    Xs, Ls = [], []
    for s in seeds:
        pos, mass, eps = training_snapshot(s, n)
        X, lab, _, _ = label_snapshot(pos, mass, eps)
        Xs.append(X)
        Ls.append(lab)
        if log:
            log(f"[learn] snapshot seed={s} n={n} groups={len(lab)} mean label={float(lab.mean()):.3f}")
    return torch.cat(Xs), torch.cat(Ls)


def fit_norm(X):
    x = X.double().cpu().numpy()
    mu = x.mean(axis=0)
    sd = x.std(axis=0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    return np.concatenate([mu, 1.0 / sd]).astype(np.float32)


def train(X, labels, epochs=40, batch=4096, lr=3e-3, lr_end=3e-4, seed=0, log=None):
    """Fit the network with Adam on minibatches; returns (MLP, per-epoch mean loss)."""
    net = bh.MLP(init_params(seed), fit_norm(X))
    t = ((labels - 0.2) / 0.8).contiguous()
    R = X.shape[0]
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, R // batch)
    total = epochs * steps_per_epoch
    history = []
    step = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(R).astype(np.int32), device="cuda")
        losses = []
        for b in range(steps_per_epoch):
            g = net.grad(X, t, perm[b * batch:(b + 1) * batch])
            # cosine decay from lr to lr_end
            lr_s = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * step / max(1, total - 1)))
            net.adam(g, lr_s)
            losses.append(g[-1:])
            step += 1
        history.append(float(torch.cat(losses).mean().item()))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"[learn] epoch {ep} loss {history[-1]:.5f}")
    return net, history


def save_net(path, net, info):
    """Writes the network's FP32 parameters and normalisation (exactly: every FP32 value is a JSON
    number that converts back to itself) with a description of its training."""
    rec = {"format": WEIGHTS_FORMAT, "n_param": int(net.params.numel()),
           "params": [float(x) for x in net.params.cpu().numpy()],
           "norm": [float(x) for x in net.norm.cpu().numpy()], "info": info}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f)
    os.replace(tmp, path)


def load_net(path=DEFAULT_WEIGHTS, device="cuda"):
    """(MLP, info) from a file written by save_net."""
    with open(path) as f:
        rec = json.load(f)
    if rec.get("format") != WEIGHTS_FORMAT or len(rec["params"]) != N_PARAM or len(rec["norm"]) != 16:
        raise ValueError(f"{path}: not a {WEIGHTS_FORMAT} weight file")
    return bh.MLP(np.asarray(rec["params"], np.float32), np.asarray(rec["norm"], np.float32), device), rec["info"]


def scaled_theta(raw, alpha, beta, cap=1.15):
    """theta_g = min(alpha raw_g^beta, cap): the network's theta with one global scale alpha and a
    shrink exponent beta <= 1 (beta < 1 pulls the per-group values toward their geometric mean,
    which pays when the predictions are noisy)."""
    return torch.clamp(alpha * raw.double() ** beta, max=cap).float().contiguous()


def rms_error(acc, a_ref, targets):
    """RMS of |a - a_ref| / |a_ref| over the sampled targets (a_ref float64 [len(targets), 3])."""
    return metrics.rms_rel_err(acc[targets], a_ref)


def bisect(f, lo, hi, target, rel=0.02, iters=40):
    """Largest x in [lo, hi] with f(x) <= target, f increasing; stops within rel of the target.
    Returns (x, f(x))."""
    flo = f(lo)
    if flo > target:
        return lo, flo
    fhi = f(hi)
    if fhi <= target:
        return hi, fhi
    best = (lo, flo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if fm <= target:
            lo, best = mid, (mid, fm)
            if fm >= target * (1 - rel):
                break
        else:
            hi = mid
    return best
