"""CPU FP64 oracle of the learned opening parameter.  TEST INFRASTRUCTURE.

Only the test suite may import this module (like the rest of ``oracle/``); the
GPU library never does.  The paper has no learned component: what follows is
the definition the GPU path is held to, written plainly in numpy.

* ``features``  -- 8 scale-free descriptors of each walk group of 64
  particles (group g = the Morton positions order[64g, 64g+64) of a walk order,
  by default the Morton order itself):
    0  log2(h / h_typ): AABB half-width h against the half-width a group of 64
       would have in a uniform cube of the same N, h_typ = L (64/N)^(1/3) / 2
    1  |centre of mass - centre of mass of c| / l_c, c the smallest tree cell
       holding the whole group (the cell of the range [min, max] of its Morton
       positions), l_c its side
    2  |centre of mass - centre of mass of a| / l_a, a the ancestor of c three
       levels up (or the root)
    3  mass-weighted RMS radius about the group's centre of mass, over h
    4  |centre of mass - AABB centre| / h
    5  log10(rho_c / rho_mean): density M/l^3 of the smallest tree cell
       holding the whole group, against M_tot / L^3
    6  log10(rho_p / rho_mean): the same for that cell's parent
    7  log2(l_c / h): size of that cell against the group's half-width
  h is floored at L 2^-22 (coincident particles), masses at 1e-300.
* ``forward`` / ``backward`` -- the MLP 8 -> 64 -> 64 -> 1 with tanh-form
  GELU: x' = bf16((x - mu) * inv_sd); h1 = bf16(gelu(W1 x' + b1));
  h2 = bf16(gelu(W2 h1 + b2)); z = w3 . h2 + b3; theta = 0.2 + 0.8 sigmoid(z).
  Weights enter as bf16(W), biases unrounded.  The loss of a batch is
  mean((sigmoid(z) - t)^2) with t = (theta* - 0.2) / 0.8.  The backward pass
  rounds the two hidden-layer error signals to bf16 where the GPU feeds them
  to its matrix cores: dW2 = bf16(dpre2)^T h1, dh1 = bf16(dpre2) W2b,
  dW1 = bf16(dpre1)^T x'.  With ``emulate=False`` nothing is rounded (the
  plain FP64 function, for finite-difference checks).
* ``adam``      -- one Adam step (Kingma & Ba 2015) on the flat parameters.
* ``bf16``      -- round to the nearest bfloat16, ties to even, of the FP32
  rounding of x (the GPU rounds FP32 values).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 8, 64
LAYOUT = {"W1": (0, (N_H, N_IN)), "b1": (512, (N_H,)), "W2": (576, (N_H, N_H)), "b2": (4672, (N_H,)),
          "w3": (4736, (N_H,)), "b3": (4800, (1,))}
N_PARAM = 4801
THETA_LO, THETA_SPAN = 0.2, 0.8
GELU_C = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


def unpack(P):
    P = np.asarray(P, np.float64)
    return {k: P[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in LAYOUT.items()}


def pack(d):
    P = np.zeros(N_PARAM)
    for k, (o, s) in LAYOUT.items():
        P[o:o + int(np.prod(s))] = np.asarray(d[k], np.float64).ravel()
    return P


def bf16(x):
    x32 = np.ascontiguousarray(np.asarray(x, np.float64), dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(x32), np.nan, out)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


def gelu_grad(x):
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def _q(emulate):
    return bf16 if emulate else (lambda v: np.asarray(v, np.float64))


def forward(P, X, mu, inv_sd, emulate=True):
    """Hidden states and outputs for rows X [R, 8] (see the module docstring)."""
    q = _q(emulate)
    p = unpack(P)
    X = np.asarray(X, np.float64)
    xb = q((X - np.asarray(mu, np.float64)) * np.asarray(inv_sd, np.float64))
    W1, W2, w3 = q(p["W1"]), q(p["W2"]), q(p["w3"])
    pre1 = xb @ W1.T + p["b1"]
    h1 = q(gelu(pre1))
    pre2 = h1 @ W2.T + p["b2"]
    h2 = q(gelu(pre2))
    z = h2 @ w3 + p["b3"][0]
    y = sigmoid(z)
    return dict(xb=xb, W1=W1, W2=W2, w3=w3, pre1=pre1, h1=h1, pre2=pre2, h2=h2, z=z, y=y,
                theta=THETA_LO + THETA_SPAN * y)


def loss_and_grad(P, X, t, mu, inv_sd, emulate=True):
    """Batch loss mean((y - t)^2) and its gradient with respect to the flat parameters."""
    q = _q(emulate)
    f = forward(P, X, mu, inv_sd, emulate)
    B = len(X)
    e = f["y"] - np.asarray(t, np.float64)
    loss = float(np.mean(e * e))
    dz = (2.0 / B) * e * f["y"] * (1.0 - f["y"])
    g = {"w3": f["h2"].T @ dz, "b3": np.array([dz.sum()])}
    dpre2 = np.outer(dz, f["w3"]) * gelu_grad(f["pre2"])
    g["b2"] = dpre2.sum(axis=0)
    dp2 = q(dpre2)
    g["W2"] = dp2.T @ f["h1"]
    dpre1 = (dp2 @ f["W2"]) * gelu_grad(f["pre1"])
    g["b1"] = dpre1.sum(axis=0)
    g["W1"] = q(dpre1).T @ f["xb"]
    return loss, pack(g)


def adam(P, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns the new (P, m, v).  ``step`` counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """Deterministic initial weights: uniform(+-1/sqrt(fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.uniform(-1, 1, (N_H, N_IN)) / np.sqrt(N_IN), "b1": np.zeros(N_H),
         "W2": rng.uniform(-1, 1, (N_H, N_H)) / np.sqrt(N_H), "b2": np.zeros(N_H),
         "w3": rng.uniform(-1, 1, N_H) / np.sqrt(N_H), "b3": np.zeros(1)}
    return pack(d)


def containing_path(tree, a, b):
    """Root-to-leaf path of ``tree`` (oracle.Tree) down to the deepest node whose particle range
    holds Morton positions [a, b)."""
    path = [0]
    while not tree.leaf[path[-1]]:
        c = path[-1]
        ch, nxt, found = c + 1, tree.next[c], -1
        while ch < nxt:
            if tree.first[ch] <= a and tree.first[ch] + tree.count[ch] >= b:
                found = ch
                break
            ch = tree.next[ch]
        if found < 0:
            break
        path.append(found)
    return path


def containing_cell(tree, a, b):
    """The deepest node holding [a, b) and its parent (the root is its own parent)."""
    path = containing_path(tree, a, b)
    return path[-1], path[-2] if len(path) > 1 else path[-1]


def features(tree, pos, mass, order=None):
    """Features [G, 8] of the walk groups of ``tree`` built from pos [n,3], mass [n] (float64);
    order: Morton positions in walk order (None: the Morton order)."""
    n = len(pos)
    order = np.arange(n) if order is None else np.asarray(order, np.int64)
    ps = np.asarray(pos, np.float64)[tree.perm][order]
    ms = np.asarray(mass, np.float64)[tree.perm][order]
    L = tree.L
    Mtot = float(tree.M[0]) if len(tree.M) else 0.0
    rho_mean = max(Mtot, 1e-300) / L ** 3
    h_typ = 0.5 * L * (64.0 / n) ** (1.0 / 3.0)
    G = (n + 63) // 64
    X = np.zeros((G, 8))
    for g in range(G):
        a, b = 64 * g, min(n, 64 * g + 64)
        p, m = ps[a:b], ms[a:b]
        lo, hi = p.min(axis=0), p.max(axis=0)
        h = max(float(np.max(hi - lo)) * 0.5, L * 2.0 ** -22)
        gc = 0.5 * (lo + hi)
        M = float(m.sum())
        com = (m[:, None] * p).sum(axis=0) / M if M > 0 else gc
        r2 = ((p - com) ** 2).sum(axis=1)
        rms = np.sqrt(float((m * r2).sum()) / M) if M > 0 else 0.0
        path = containing_path(tree, int(order[a:b].min()), int(order[a:b].max()) + 1)
        c = path[-1]
        par = path[-2] if len(path) > 1 else c
        anc = path[-4] if len(path) > 3 else path[0]
        X[g, 0] = np.log2(h / h_typ)
        X[g, 1] = np.sqrt(float(((com - tree.com[c]) ** 2).sum())) / tree.l[c]
        X[g, 2] = np.sqrt(float(((com - tree.com[anc]) ** 2).sum())) / tree.l[anc]
        X[g, 3] = rms / h
        X[g, 4] = np.sqrt(float(((com - gc) ** 2).sum())) / h
        X[g, 5] = np.log10(max(tree.M[c], 1e-300) / tree.l[c] ** 3 / rho_mean)
        X[g, 6] = np.log10(max(tree.M[par], 1e-300) / tree.l[par] ** 3 / rho_mean)
        X[g, 7] = np.log2(tree.l[c] / h)
    return X


def group_rms(acc, acc_ref, perm, order=None):
    """Per walk group (as in features): RMS over its particles of |a - a_ref| / |a_ref|
    (caller-order inputs).

    The relative error of Eq. (4) is undefined where a_ref = 0: such particles are left out of
    their group's mean, and a group with none left has RMS 0."""
    sel = np.asarray(perm) if order is None else np.asarray(perm)[np.asarray(order, np.int64)]
    acc = np.asarray(acc, np.float64)[sel]
    ref = np.asarray(acc_ref, np.float64)[sel]
    den = np.linalg.norm(ref, axis=1)
    ok = den > 0
    d = np.zeros(len(den))
    d[ok] = np.linalg.norm(acc - ref, axis=1)[ok] / den[ok]
    n = len(d)
    G = (n + 63) // 64
    out = np.zeros(G)
    for g in range(G):
        sl = slice(64 * g, min(n, 64 * g + 64))
        s = d[sl][ok[sl]]
        out[g] = np.sqrt(np.mean(s * s)) if len(s) else 0.0
    return out
