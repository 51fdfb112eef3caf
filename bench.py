"""Benchmark of the tree-force hot path on one MI355X.

One step = build the tree (bbox, Morton keys, radix sort, topology, FP64
moments) + the force walk for every particle, on the 4,194,304-particle clumpy
field (25% uniform in the unit cube + 64 Plummer clumps, a = 0.01), FP32
inputs, eps = 1e-4, at the opening parameter that reaches an RMS relative
force error <= 1e-3 against the direct sum (checked on 65,536 sampled targets
with the GPU FP64 direct sum, outside the timed region).

Prints one JSON line.  ``value`` = particle interactions per second of the
whole step (interactions counted by the instrumented walk, identical lists).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

METRIC = "particle-interactions/s and forces/s at RMS rel force err 1e-3, N=4M, 1 GPU"
FLOPS_PER_INTERACTION = 38          # the paper's conventional count (Sec. 3)
# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s for FP64 and for
# unpacked FP32 -- the instructions the walk issues (FP64 offsets, tests and sums, unpacked FP32
# terms); packed FP32 doubles the FP32 rate to 157.3 TFLOP/s, which this code does not use.
PEAK_VALU_TFLOPS = 78.6
PEAK_PACKED_FP32_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(workload, theta, kind="walk", key="theta"):
    """HBM bytes per launch of a walk (kind "walk", at theta) or of the neighbour walk (kind "nbr",
    at the radius: key "radius") from the committed counter summary, or None.

    The figure holds only for the kernel source it was counted on: the summary
    stores a digest of the kernel's sources and is ignored once they changed.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for p in rec["sources"]:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    if h.hexdigest() != rec["source_sha256"] or abs(rec.get(key, theta) - theta) > 1e-12:
        return None
    return rec["traffic_bytes"]


def cpu_baseline(pos32, mass32, theta, eps, seed, n_sample, n_sample_1t):
    """The FP64 CPU oracle on this host: full tree build + walk of a target sample, scaled to all
    targets; on all the threads OpenMP gives it, and on one thread (walk sample n_sample_1t; the
    tree build is serial code in both)."""
    import oracle
    from paper_1112_4539_amd import inputs
    p64 = pos32.astype(np.float64)
    m64 = mass32.astype(np.float64)
    n = len(p64)
    t0 = time.perf_counter()
    T = oracle.Tree(p64, m64)
    t1 = time.perf_counter()
    cores = oracle.num_threads()

    def walk(count, salt):
        tg = inputs.sample_targets(n, count, seed + salt)
        s0 = time.perf_counter()
        w = T.walk(theta, eps, targets=tg)
        s1 = time.perf_counter()
        inter = float(np.sum(w["n_pp"] + w["n_pc"]))
        scale = n / len(tg)
        t_total = (t1 - t0) + (s1 - s0) * scale
        return inter * scale / t_total, len(tg), s1 - s0, scale

    v, k, ws, scale = walk(n_sample, 7)
    oracle.set_num_threads(1)
    try:
        v1, k1, ws1, scale1 = walk(n_sample_1t, 8)
    finally:
        oracle.set_num_threads(cores)
    return dict(value=v, unit="interactions/s", cores=cores, kind="oracle",
                sample=f"FP64 oracle: tree build of all {n} particles ({t1 - t0:.2f} s, serial) + walk of {k} "
                       f"sampled targets ({ws:.2f} s on {cores} threads), walk time scaled by {scale:.1f} to all "
                       f"targets",
                one_thread={"value": v1, "unit": "interactions/s", "cores": 1,
                            "sample": f"same build + walk of {k1} sampled targets on 1 thread ({ws1:.2f} s), "
                                      f"scaled by {scale1:.1f}"})


def forest_bench(args, bh, inputs):
    """512 independent Plummer clusters (log-uniform N in [1024, 65536], seed 3), theta 0.5,
    eps 0.01, FP32: the whole pipeline (forest build + walk) as one captured HIP graph with the
    autotuned walk shape, against a build and a walk per cluster."""
    pos, mass, off = inputs.clusters(512, 3)
    n = len(pos)
    theta, eps = 0.5, 0.01
    dev = torch.device("cuda:0")
    gpos = torch.tensor(pos.astype(np.float32), device=dev)
    gmass = torch.tensor(mass.astype(np.float32), device=dev)
    goff = torch.tensor(off, device=dev)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((n,), dtype=torch.float32, device=dev)
    log(f"[bench] forest: {len(off) - 1} clusters, n={n}")
    F = bh.build_forest(gpos, gmass, goff)
    F.check()
    F.set_walk_config(target_order=args.target_order)
    st = F.walk_stats(theta, eps)
    inter = int(st["counts"].to(torch.int64).sum().item())
    del st
    best, tried = F.autotune(theta, eps, acc, pot, reps=2)
    log(f"[bench] autotuned walk shape {best} ({len(tried)} candidates)")
    G = F.graph(theta, eps, acc, pot)
    for _ in range(args.warmup):
        G.launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        G.launch()
    ev1.record()
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    # walk alone, autotuned shape (HIP events around the walk kernel)
    F.set_timing(True)
    wt = []
    for _ in range(args.steps):
        F.forces(theta, eps, acc, pot)
        wt.append(F.walk_time_ms())
    walk_ms = float(np.mean(wt))
    # one build and one walk per cluster, default shape
    sub = [(int(off[k]), int(off[k + 1])) for k in range(len(off) - 1)]
    ws = torch.empty(bh.workspace_bytes(int(np.max(np.diff(off))), bh.FP32), dtype=torch.uint8, device=dev)

    def per_cluster():
        # (Morton target order: for trees this small the Hilbert order's sort costs more than it saves)
        for b, e in sub:
            T = bh.Tree(gpos[b:e], gmass[b:e], workspace=ws)
            T.set_walk_config(target_order=0)
            T.forces(theta, eps, acc[b:e], pot[b:e])

    per_cluster()
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    ev0.record()
    for _ in range(reps):
        per_cluster()
    ev1.record()
    torch.cuda.synchronize()
    per_ms = ev0.elapsed_time(ev1) / reps
    line = {
        "metric": "particle-interactions/s, 512 clusters in one captured launch",
        "value": inter / (graph_ms * 1e-3), "unit": "interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": graph_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"512 Plummer clusters, N log-uniform in [1024, 65536], seed 3, n={n}, "
                               f"theta={theta}, eps={eps}, FP32",
                   "interactions_per_step": inter, "graph_ms": graph_ms, "walk_ms": walk_ms,
                   "per_cluster_ms": per_ms, "speedup_vs_per_cluster": per_ms / graph_ms,
                   "target_order": args.target_order, "autotuned": best, "candidates": tried},
    }
    print(json.dumps(line), flush=True)


def sweep_bench(args, bh, inputs):
    """Plummer N=1,048,576 (seed 1, eps 0.005): per theta in {0.3, 0.5, 0.75}, the RMS and mean
    relative force error against the FP64 direct sum on 65,536 sampled targets, interactions, and
    the walk time with targets in Hilbert order (the default), in Morton order and in the input
    (random) order; the FP64 walk
    beside it as the accuracy reference of the FP32 arithmetic."""
    from paper_1112_4539_amd import metrics
    pos, mass, spec = inputs.make("plummer1m")
    eps = spec["eps"]
    n = len(pos)
    dev = torch.device("cuda:0")
    g32 = (torch.tensor(pos.astype(np.float32), device=dev), torch.tensor(mass.astype(np.float32), device=dev))
    g64 = (g32[0].double(), g32[1].double())
    tg = torch.tensor(inputs.sample_targets(n, args.samples, spec["seed"]), device=dev)
    a_ref, _ = bh.direct(g64[0], g64[1], eps, tg)
    T32 = bh.Tree(*g32)
    T64 = bh.Tree(*g64)

    def walk_ms(T, theta, order, reps):
        T.set_walk_config(target_order=order)
        T.set_timing(True)
        ms = []
        for _ in range(reps):
            T.forces(theta, eps)
            ms.append(T.walk_time_ms())
        T.set_timing(False)
        T.set_walk_config(target_order=2)
        return min(ms)

    rows = []
    for theta in spec["thetas"]:
        st = T32.walk_stats(theta, eps)
        inter = int(st["counts"].to(torch.int64).sum().item())
        steps = int(st["group_steps"].to(torch.int64).sum().item())
        a64, _ = T64.forces(theta, eps)
        d3264 = metrics.rel_errors(st["acc"][tg], a64[tg])
        ms_m = walk_ms(T32, theta, 0, max(3, args.steps))
        ms_h = walk_ms(T32, theta, 2, max(3, args.steps))
        ms_r = walk_ms(T32, theta, 1, 2)
        ms_64 = walk_ms(T64, theta, 2, 3)
        row = dict(theta=theta, interactions=inter, mean_list=inter / n, lane_efficiency=inter / (64.0 * steps),
                   rms_rel_err=metrics.rms_rel_err(st["acc"][tg], a_ref),
                   mean_rel_err=metrics.mean_rel_err(st["acc"][tg], a_ref),
                   rms_rel_err_fp64_walk=metrics.rms_rel_err(a64[tg], a_ref),
                   max_rel_diff_fp32_vs_fp64_walk=float(d3264.max()),
                   walk_ms_morton=ms_m, walk_ms_hilbert=ms_h, walk_ms_random_order=ms_r,
                   random_over_morton=ms_r / ms_m, walk_ms_fp64=ms_64, interactions_per_s=inter / (ms_h * 1e-3))
        log(f"[bench] theta={theta}: {json.dumps(row)}")
        rows.append(row)
    line = {"metric": "per-theta force error and localized-ordering effect, Plummer N=1M",
            "value": rows[1]["interactions_per_s"], "unit": "interactions/s (theta 0.5, Hilbert target order)",
            "n_gpus": 1, "steps": args.steps, "warmup": 0, "ms_per_step": rows[1]["walk_ms_hilbert"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"Plummer sphere N={n} (a=1, truncated at 10a), seed {spec['seed']}, eps={eps}, FP32",
                       "accuracy_targets": args.samples, "thetas": rows}}
    print(json.dumps(line), flush=True)


def learned_bench(args, bh, inputs):
    """Learned per-group opening parameter against fixed theta at equal accuracy (RMS relative
    force error 1e-3 against the FP64 direct sum on 65,536 sampled targets), on the clumpy field
    N=8,388,608 (seed 4, eps 1e-4).  Two networks are trained on the GPU:
    (a) on 64 snapshots of 262,144 particles (seeds 100-163, Plummer and clumpy alternately), its
        shrink exponent picked on a held-out snapshot (seed 164);
    (b) on labels from 2048 sampled groups of each of 8 clumpy fields at the evaluation's size
        (N=8,388,608, seeds 200-207).
    Reported: interactions and walk time of the FP32 fixed-theta walk, of the FP32 walks with
    either network's theta, and of the FP64 fixed-theta walk."""
    from paper_1112_4539_amd import learn
    t0 = time.perf_counter()
    X, L = learn.build_dataset(range(100, 164), log=log)
    t1 = time.perf_counter()
    net, hist = learn.train(X, L, epochs=60, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"[bench] (a) labels {t1 - t0:.1f} s, training {t2 - t1:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    X8, L8 = learn.build_dataset_sampled(range(200, 208), 8388608, 2048, log=log)
    t3 = time.perf_counter()
    net8, hist8 = learn.train(X8, L8, epochs=80, batch=1024, log=log)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    log(f"[bench] (b) labels {t3 - t2:.1f} s, training {t4 - t3:.1f} s, loss {hist8[0]:.4f} -> {hist8[-1]:.4f}")
    target = learn.TARGET

    def evaluate(pos, mass, eps, n_targets, seed, nets, with_fp64):
        """nets: {name: (network, [shrink exponents])}."""
        dev = torch.device("cuda:0")
        g32 = (torch.tensor(pos.astype(np.float32), device=dev), torch.tensor(mass.astype(np.float32), device=dev))
        n = len(pos)
        tg = torch.tensor(inputs.sample_targets(n, n_targets, seed), device=dev)
        a_ref, _ = bh.direct(g32[0].double(), g32[1].double(), eps, tg)
        T = bh.Tree(*g32)
        T.set_walk_config(target_order=args.target_order)
        X = T.features()

        def run(T, theta=None, tgrp=None, reps=3):
            st = T.walk_stats(theta if theta else 0.5, eps, theta_group=tgrp)
            inter = int(st["counts"].to(torch.int64).sum().item())
            T.set_timing(True)
            ms = []
            for _ in range(reps):
                T.forces(theta if theta else 0.5, eps, theta_group=tgrp)
                ms.append(T.walk_time_ms())
            T.set_timing(False)
            return inter, min(ms)

        thf, ef = learn.bisect(lambda th: learn.rms_error(T.forces(th, eps)[0], a_ref, tg), 0.1, 1.1, target)
        i_f, ms_f = run(T, theta=thf)
        out = {"fixed_fp32": dict(theta=thf, rms=ef, interactions=i_f, walk_ms=ms_f)}
        for name, (nw, betas) in nets.items():
            raw = nw.infer(X, alpha=1.0, fallback=0.5)
            for beta in betas:
                def rms_l(alpha, beta=beta):
                    a, _ = T.forces(0.5, eps, theta_group=learn.scaled_theta(raw, alpha, beta))
                    return learn.rms_error(a, a_ref, tg)
                al, el = learn.bisect(rms_l, 0.05, 4.0, target)
                tgrp = learn.scaled_theta(raw, al, beta)
                i_l, ms_l = run(T, tgrp=tgrp)
                out[f"{name}_beta{beta}"] = dict(alpha=al, beta=beta, rms=el, interactions=i_l, walk_ms=ms_l,
                                                 theta_mean=float(tgrp.mean()), interactions_vs_fixed=i_l / i_f,
                                                 walk_ms_vs_fixed=ms_l / ms_f)
        if with_fp64:
            T64 = bh.Tree(g32[0].double(), g32[1].double())
            T64.set_walk_config(target_order=args.target_order)
            th64, e64 = learn.bisect(lambda th: learn.rms_error(T64.forces(th, eps)[0], a_ref, tg), 0.1, 1.1, target)
            i64, ms64 = run(T64, theta=th64)
            out["fixed_fp64"] = dict(theta=th64, rms=e64, interactions=i64, walk_ms=ms64)
        return out

    pos, mass, eps = learn.training_snapshot(164)
    held = evaluate(pos, mass, eps, 65536, 164, {"learned": (net, (1.0, 0.8, 0.6, 0.4))}, False)
    beta = min((v["interactions"], v["beta"]) for k, v in held.items() if k.startswith("learned"))[1]
    log(f"[bench] held-out snapshot: {json.dumps(held)}; shrink exponent {beta}")
    pos, mass, spec = inputs.make("clumpy8m")
    res = evaluate(pos, mass, spec["eps"], args.samples, spec["seed"],
                   {"learned": (net, (beta,)), "learned8m": (net8, (1.0,))}, True)
    log(f"[bench] clumpy 8M: {json.dumps(res)}")
    n = len(pos)
    lr = res["learned8m_beta1.0"]
    line = {"metric": "forces/s at RMS rel force err 1e-3, learned per-group theta (clumpy N=8M)",
            "value": n / (lr["walk_ms"] * 1e-3), "unit": "forces/s (walk)", "n_gpus": 1, "steps": 3,
            "warmup": 0, "ms_per_step": lr["walk_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"clumpy field N={n}, seed {spec['seed']}, eps={spec['eps']}; network trained "
                                   f"on 2048 sampled groups of each of 8 clumpy fields N=8388608 (seeds 200-207)",
                       "train_rows": int(L8.shape[0]), "train_loss": [hist8[0], hist8[-1]],
                       "label_s": t3 - t2, "train_s": t4 - t3,
                       "small_snapshot_network": {"train_rows": int(L.shape[0]), "train_loss": [hist[0], hist[-1]],
                                                  "label_s": t1 - t0, "train_s": t2 - t1, "shrink_exponent": beta,
                                                  "heldout": held},
                       "eval": res,
                       "forces_per_s": {k: n / (v["walk_ms"] * 1e-3) for k, v in res.items()}}}
    print(json.dumps(line), flush=True)


def cube_bench(args, bh, inputs):
    """The paper's uniform-cube run for context: N = 1,048,576 particles uniform in the unit cube
    (seed 5, equal masses), theta = 0.6, FP32; the whole step (build + walk) is timed.  The
    paper's softening for this run is not stated; eps = 1e-3 here."""
    n, theta, eps = 1 << 20, 0.6, 1e-3
    rng = np.random.default_rng(5)
    pos = rng.random((n, 3))
    dev = torch.device("cuda:0")
    gpos = torch.tensor(pos.astype(np.float32), device=dev)
    gmass = torch.full((n,), 1.0 / n, dtype=torch.float32, device=dev)
    ws = torch.empty(bh.workspace_bytes(n, bh.FP32), dtype=torch.uint8, device=dev)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((n,), dtype=torch.float32, device=dev)
    T = bh.Tree(gpos, gmass, workspace=ws)
    inter = int(T.walk_stats(theta, eps)["counts"].to(torch.int64).sum().item())
    for _ in range(args.warmup):
        bh.Tree(gpos, gmass, workspace=ws).forces(theta, eps, acc, pot)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        bh.Tree(gpos, gmass, workspace=ws).forces(theta, eps, acc, pot)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    line = {"metric": "forces/s, uniform cube N=1M, theta 0.6 (the paper's context run)",
            "value": n / (ms * 1e-3), "unit": "forces/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"uniform cube N={n}, seed 5, theta={theta}, eps={eps}, FP32",
                       "interactions_per_step": inter, "interactions_per_s": inter / (ms * 1e-3)}}
    print(json.dumps(line), flush=True)


def quad_steps(args, bh, inputs, gpos, gmass, ws, acc, pot, eps, n, ref):
    """The same step with order-2 cell terms (quadrupole) at --quad-theta: build + second moments +
    walk, timed like the headline; RMS error on the same sampled targets; interactions counted."""
    theta = args.quad_theta

    def make():
        T = bh.Tree(gpos, gmass, workspace=ws)
        T.set_walk_config(args.waves_per_block, args.xcd_chunk, args.target_order, args.lds_share, args.persistent,
                          args.targets_per_lane)
        T.set_order(2)
        return T

    for _ in range(args.warmup):
        make().forces(theta, eps, acc=acc, pot=pot)
    T = make()
    st = T.walk_stats(theta, eps)
    inter = int(st["counts"].to(torch.int64).sum().item())
    del st, T
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    trees = []
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        T = make()
        T.set_timing(True)
        T.forces(theta, eps, acc=acc, pot=pot)
        trees.append(T)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    walk = float(np.mean([T.walk_time_ms() for T in trees]))
    del trees
    rms = None
    if ref is not None:
        from paper_1112_4539_amd import metrics
        T = make()
        a, _ = T.forces(theta, eps, acc=acc, pot=pot)
        rms = metrics.rms_rel_err(a[ref[0]], ref[1])
    log(f"[bench] quadrupole theta={theta}: ms/step={ms:.3f} walk {walk:.3f} ms, interactions {inter}, RMS {rms}")
    return {"theta": theta, "rms_rel_force_err": rms, "interactions_per_step": inter, "ms_per_step": ms,
            "walk_ms": walk, "forces_per_s": n / (ms * 1e-3), "interactions_per_s": inter / (ms * 1e-3)}


def learned_headline(args, bh, gpos, gmass, eps, n, ref, fixed):
    """The shipped opening-parameter network on the headline field, outside the timed region: the
    per-group theta of the network times one scale alpha, and one fixed theta, each bisected to the
    RMS error target on the same sampled targets; interactions and walk time (median of 5 launches)
    of the learned FP32 walk against the fixed-theta FP32 and FP64 walks."""
    from paper_1112_4539_amd import learn
    if not os.path.exists(args.weights):
        return {"weights": None, "note": f"no weight file at {args.weights}"}
    net, info = learn.load_net(args.weights)
    tg, a_ref = ref
    T = bh.Tree(gpos, gmass)
    T.set_walk_config(args.waves_per_block, args.xcd_chunk, args.target_order, args.lds_share, args.persistent,
                      args.targets_per_lane)
    raw = net.infer(T.features(), alpha=1.0, fallback=0.5)

    def per_group(alpha):
        return {"theta_group": learn.scaled_theta(raw, alpha, 1.0)}

    def rms(kw):
        return learn.rms_error(T.forces(0.5, eps, **kw)[0], a_ref, tg)

    def timed(T, reps, theta=0.5, **kw):
        T.set_timing(True)
        ms = []
        for _ in range(reps):
            T.forces(theta, eps, **kw)
            ms.append(T.walk_time_ms())
        T.set_timing(False)
        return float(np.median(ms))

    def count(theta=0.5, **kw):
        st = T.walk_stats(theta, eps, **kw)
        return int(st["counts"].to(torch.int64).sum().item())

    alpha, err = learn.bisect(lambda a: rms(per_group(a)), 0.05, 4.0, learn.TARGET)
    kw_g = per_group(alpha)
    # the fixed theta bisected to the same target (the headline's theta is the largest on a 0.05
    # grid, a little below it)
    thf, ef = learn.bisect(lambda th: learn.rms_error(T.forces(th, eps)[0], a_ref, tg), 0.1, 1.1, learn.TARGET)
    inter, inter_f = count(**kw_g), count(thf)
    ms_l, ms_f = timed(T, 5, **kw_g), timed(T, 5, thf)
    del T
    T64 = bh.Tree(gpos.double(), gmass.double())
    T64.set_walk_config(target_order=args.target_order)
    a64, _ = T64.forces(thf, eps)
    rms64 = learn.rms_error(a64, a_ref, tg)
    ms64 = timed(T64, 3, thf)
    del T64, a64
    out = {"weights": os.path.relpath(args.weights, ROOT), "trained_on": info.get("fields"),
           "alpha": alpha, "theta_mean": float(kw_g["theta_group"].mean()), "rms_rel_force_err": err,
           "interactions": inter, "walk_ms": ms_l,
           "interactions_vs_fixed": inter / inter_f, "walk_ms_vs_fixed": ms_l / ms_f,
           "forces_per_s_walk": n / (ms_l * 1e-3),
           "fixed_fp32": {"theta": thf, "rms_rel_force_err": ef, "interactions": inter_f, "walk_ms": ms_f},
           "fixed_fp64": {"theta": thf, "rms_rel_force_err": rms64, "walk_ms": ms64},
           "walk_ms_vs_fixed_fp64": ms_l / ms64,
           "headline_theta": {"theta": args.theta, "rms_rel_force_err": fixed["rms"],
                              "interactions": fixed["interactions"], "walk_ms": fixed["walk_ms"]}}
    log(f"[bench] learned theta: {json.dumps(out)}")
    return out


# Algorithmic work of one neighbour pair (i, j within r): the distance test, 8 flops (three
# differences, three squares, two sums), and the density term, 12 (the square root, q = r/h, the
# spline's cubic in q, the mass product and the sum).
FLOPS_PER_NEIGHBOUR_PAIR = 20


def neighbours_bench(args, bh, inputs):
    """The general tree walk of Sec. 4.3 as a neighbour search with the SPH density, on the clumpy
    field N=4,194,304 (FP32, the force headline's field) at radius --radius: each call copies the
    nodes with their skip radii and walks every particle.  value = neighbour pairs per second."""
    pos, mass, spec = inputs.make("clumpy4m")
    n = len(pos)
    r = args.radius
    f64 = args.nbr_prec == "fp64"
    ft = np.float64 if f64 else np.float32
    log(f"[bench] neighbours clumpy4m r={r} {args.nbr_prec}")
    dev = torch.device("cuda:0")
    gpos = torch.tensor(pos.astype(ft), device=dev)
    gmass = torch.tensor(mass.astype(ft), device=dev)
    T = bh.Tree(gpos, gmass)
    out = T.neighbours(r)
    cnt = out["count"].to(torch.int64)
    pairs = int(cnt.sum().item())
    for _ in range(args.warmup):
        T.neighbours(r)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        T.neighbours(r)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    # the walk kernel alone, bracketed by the tree's HIP events on the stream it runs on
    T.set_timing(True)
    kms = []
    for _ in range(args.steps):
        T.neighbours(r)
        kms.append(T.walk_time_ms())
    T.set_timing(False)
    kernel_ms = float(np.mean(kms))
    achieved = FLOPS_PER_NEIGHBOUR_PAIR * pairs / (kernel_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        import oracle
        p64 = pos.astype(ft).astype(np.float64)
        m64 = mass.astype(ft).astype(np.float64)
        t0 = time.perf_counter()
        O = oracle.Tree(p64, m64)
        t1 = time.perf_counter()
        w = O.neighbours(r)
        t2 = time.perf_counter()
        cpu = {"value": float(np.sum(w["count"])) / (t2 - t0), "unit": "neighbour pairs/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"the whole workload once in FP64: tree build ({t1 - t0:.2f} s) + neighbour walk with "
                         f"the density of all {n} targets ({t2 - t1:.2f} s)"}
        log(f"[bench] oracle pairs {int(np.sum(w['count']))} vs kernel {pairs}")
    line = {"metric": f"neighbour pairs/s with the SPH density, clumpy N={n}, r={r}" + (", FP64" if f64 else ""),
            "value": pairs / (ms * 1e-3), "unit": "neighbour pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if f64 else "f32+f64", "data": "synthetic",
            "config": {"workload": f"clumpy field N={n}, seed {spec['seed']}, {'FP64' if f64 else 'FP32'}, radius {r}, "
                                   "SPH density (M4, h = r/2)",
                       "pairs_per_step": pairs, "mean_neighbours": pairs / n, "max_neighbours": int(cnt.max().item()),
                       "no_neighbour_share": float((cnt == 0).double().mean().item()),
                       "walk_kernel_ms": kernel_ms},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_VALU_TFLOPS,
                         "traffic": None if f64 else measured_traffic("clumpy4m", r, kind="nbr", key="radius"),
                         "kernel": f"bh::k_nbr<{'true' if f64 else 'false'}, false>",
                         "flops_per_unit": FLOPS_PER_NEIGHBOUR_PAIR,
                         "units_per_launch": pairs,
                         "peak_note": "FP64 and unpacked FP32 vector rate; the search is bound by its dependent "
                                      "node-record loads and instruction issue, not by arithmetic"},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def leapfrog_bench(args, bh, inputs):
    """The time loop on the clumpy field N=4,194,304 (FP32, theta --theta, eps 1e-4): kick-drift-kick
    leapfrog steps with a tree rebuild each step, with the state kept in the caller's (random) order
    and with it permuted into each new tree's Morton order (Sec. 5: the order comes for free)."""
    pos, mass, spec = inputs.make("clumpy4m")
    eps, theta, dt = spec["eps"], args.theta, 1e-5
    n = len(pos)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(9)
    vel0 = 0.01 * rng.normal(size=pos.shape)
    ws = torch.empty(bh.workspace_bytes(n, bh.FP32), dtype=torch.uint8, device=dev)
    res = {}
    for reorder in (False, True):
        P = torch.tensor(pos.astype(np.float32), device=dev)
        V = torch.tensor(vel0.astype(np.float32), device=dev)
        M = torch.tensor(mass.astype(np.float32), device=dev)
        A, U = bh.Tree(P, M, workspace=ws).forces(theta, eps)
        A, U = A.clone(), U.clone()
        for _ in range(args.warmup):
            bh.leapfrog_step(P, V, M, A, U, dt, theta, eps, reorder=reorder, workspace=ws)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            bh.leapfrog_step(P, V, M, A, U, dt, theta, eps, reorder=reorder, workspace=ws)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        # build alone on the state as it now stands (caller order, or the last Morton order)
        ev0.record()
        for _ in range(args.steps):
            bh.Tree(P, M, workspace=ws)
        ev1.record()
        torch.cuda.synchronize()
        res["morton_reorder" if reorder else "caller_order"] = {
            "ms_per_step": ms, "steps_per_s": 1e3 / ms, "build_ms": ev0.elapsed_time(ev1) / args.steps}
        log(f"[bench] leapfrog reorder={reorder}: {res}")
    line = {"metric": "leapfrog steps/s (build + walk + kicks each step), clumpy N=4M",
            "value": res["morton_reorder"]["steps_per_s"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["morton_reorder"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"clumpy field N={n}, seed {spec['seed']}, eps={eps}, theta={theta}, dt={dt}, "
                                   "FP32 state, velocities N(0, 0.01)", "modes": res}}
    print(json.dumps(line), flush=True)


def walk_only(args, bh, inputs):
    """One build and WALK_ONLY force walks of a named workload, nothing else: the command that
    the rocprofv3 counter and trace summaries are taken from (target order, expansion order and
    theta as given).  Prints the interactions of one walk."""
    pos, mass, spec = inputs.make(args.workload)
    dev = torch.device("cuda:0")
    gpos = torch.tensor(pos.astype(np.float32), device=dev)
    gmass = torch.tensor(mass.astype(np.float32), device=dev)
    T = bh.Tree(gpos, gmass)
    T.set_walk_config(args.waves_per_block, args.xcd_chunk, args.target_order, args.lds_share, args.persistent,
                      args.targets_per_lane)
    T.set_order(args.order)
    tgrp = None
    if args.theta_group == "uniform":
        # theta per walk group, every group at --theta (the fixed walk's lists, the per-group step)
        tgrp = torch.full((T.n_groups,), args.theta, dtype=torch.float32, device=dev)
    elif args.theta_group == "learned":
        from paper_1112_4539_amd import learn
        net, _ = learn.load_net(args.weights)
        tgrp = learn.scaled_theta(net.infer(T.features(), alpha=1.0, fallback=0.5), args.alpha, 1.0)
    for _ in range(args.walk_only):
        T.forces(args.theta, spec["eps"], theta_group=tgrp)
    torch.cuda.synchronize()
    log(f"[bench] walk-only: {args.workload} n={len(pos)} theta={args.theta} target_order={args.target_order} "
        f"order={args.order} theta_group={args.theta_group}: {args.walk_only} walks")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clumpy4m")
    ap.add_argument("--theta", type=float, default=0.35)
    ap.add_argument("--samples", type=int, default=65536, help="targets of the accuracy check")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-theta evaluation")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1112_4539_amd", "weights",
                                                      "theta_clumpy4m.json"),
                    help="network for the learned-theta evaluation of the headline field")
    ap.add_argument("--cpu-sample", type=int, default=262144)
    ap.add_argument("--cpu-sample-1t", type=int, default=16384, help="walk sample of the one-thread CPU figure")
    ap.add_argument("--waves-per-block", type=int, default=1)
    ap.add_argument("--xcd-chunk", type=int, default=-1)
    ap.add_argument("--target-order", type=int, default=2)
    ap.add_argument("--lds-share", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--targets-per-lane", type=int, default=1)
    ap.add_argument("--order", type=int, default=1, help="cell terms: 1 monopole, 2 with the quadrupole")
    ap.add_argument("--quad-theta", type=float, default=0.59,
                    help="also time the quadrupole step at this theta (0: skip)")
    ap.add_argument("--radius", type=float, default=2e-3, help="neighbours workload: search radius")
    ap.add_argument("--nbr-prec", choices=("fp32", "fp64"), default="fp32", help="neighbours workload: tree precision")
    ap.add_argument("--theta-group", choices=("none", "uniform", "learned"), default="none",
                    help="walk-only: theta per walk group (every group at --theta, or the shipped network's "
                         "theta times --alpha)")
    ap.add_argument("--alpha", type=float, default=0.89, help="walk-only, learned theta: the network's scale")
    ap.add_argument("--walk-only", type=int, default=0, metavar="K",
                    help="only build once and run K force walks of --workload (for profiler runs)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="first run three plain device copies of MIB MiB (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import paper_1112_4539_amd as bh
    from paper_1112_4539_amd import inputs
    from paper_1112_4539_amd import metrics

    if args.copy_calib > 0:
        # a plain copy of known size: reads and writes exactly MIB MiB each
        src = torch.ones(args.copy_calib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] copy calibration: 3 x {args.copy_calib} MiB")

    if args.workload == "clusters512":
        return forest_bench(args, bh, inputs)
    if args.walk_only:
        return walk_only(args, bh, inputs)
    if args.workload == "plummer1m":
        return sweep_bench(args, bh, inputs)
    if args.workload == "learned":
        return learned_bench(args, bh, inputs)
    if args.workload == "cube1m":
        return cube_bench(args, bh, inputs)
    if args.workload == "neighbours":
        return neighbours_bench(args, bh, inputs)
    if args.workload == "leapfrog":
        return leapfrog_bench(args, bh, inputs)

    pos, mass, spec = inputs.make(args.workload)
    eps = spec["eps"]
    n = len(pos)
    pos32 = pos.astype(np.float32)
    mass32 = mass.astype(np.float32)
    dev = torch.device("cuda:0")
    gpos = torch.tensor(pos32, device=dev)
    gmass = torch.tensor(mass32, device=dev)
    ws = torch.empty(bh.workspace_bytes(n, bh.FP32), dtype=torch.uint8, device=dev)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty((n,), dtype=torch.float32, device=dev)
    log(f"[bench] workload={args.workload} n={n} theta={args.theta} eps={eps}")

    def step():
        T = bh.Tree(gpos, gmass, workspace=ws)
        T.set_walk_config(args.waves_per_block, args.xcd_chunk, args.target_order, args.lds_share,
                          args.persistent, args.targets_per_lane)
        T.forces(args.theta, eps, acc=acc, pot=pot)
        return T

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # interaction count of one step (the instrumented walk meets the same lists)
    T = bh.Tree(gpos, gmass, workspace=ws)
    T.check()
    st = T.walk_stats(args.theta, eps)
    counts = st["counts"].to(torch.int64)
    inter = int(counts.sum().item())
    n_pp = int(counts[:, 0].sum().item())
    tstats = T.stats()
    del st, T
    torch.cuda.synchronize()
    log(f"[bench] interactions/step={inter} nodes={tstats['n_nodes']}")

    # timed steps
    walk_ms = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        T = bh.Tree(gpos, gmass, workspace=ws)
        T.set_walk_config(args.waves_per_block, args.xcd_chunk, args.target_order, args.lds_share,
                          args.persistent, args.targets_per_lane)
        T.set_timing(True)
        T.forces(args.theta, eps, acc=acc, pot=pot)
        walk_ms.append(T)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    wall_ms = (t1 - t0) * 1e3 / args.steps
    walk = [T.walk_time_ms() for T in walk_ms]
    del walk_ms
    walk_avg = float(np.mean(walk))
    log(f"[bench] ms/step={ms_step:.3f} (wall {wall_ms:.3f})  walk kernel {walk_avg:.3f} ms")

    # build alone
    ev0.record()
    for _ in range(args.steps):
        bh.Tree(gpos, gmass, workspace=ws)
    ev1.record()
    torch.cuda.synchronize()
    build_ms = ev0.elapsed_time(ev1) / args.steps

    rms = None
    if not args.no_accuracy:
        tg = torch.tensor(inputs.sample_targets(n, args.samples, spec["seed"]), device=dev)
        a_ref, _ = bh.direct(gpos.double(), gmass.double(), eps, tg)
        T = bh.Tree(gpos, gmass, workspace=ws)
        a, _ = T.forces(args.theta, eps, acc=acc, pot=pot)
        rms = metrics.rms_rel_err(a[tg], a_ref)
        log(f"[bench] RMS rel force err vs FP64 direct on {args.samples} targets: {rms:.3e}")

    learned = None
    if rms is not None and not args.no_learned:
        learned = learned_headline(args, bh, gpos, gmass, eps, n, (tg, a_ref),
                                   {"interactions": inter, "walk_ms": walk_avg, "rms": rms})

    quad = None
    if args.quad_theta > 0:
        quad = quad_steps(args, bh, inputs, gpos, gmass, ws, acc, pot, eps, n, None if rms is None else (tg, a_ref))
        quad["forces_per_s_vs_monopole"] = quad["forces_per_s"] / (n / (ms_step * 1e-3))

    value = inter / (ms_step * 1e-3)
    achieved = FLOPS_PER_INTERACTION * inter / (walk_avg * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "precision": "FP32 positions, masses and outputs; FP32 terms (r^2+eps^2 rounded once, v_rsq_f32, FP32 "
                         "products; the potential's m/r as (m/r^3)(r^2+eps^2) in its FP64 fused sum); FP64 offsets, "
                         "opening test and sums",
            "workload": f"clumpy field N={n} (25% uniform in the unit cube + 64 Plummer clumps a=0.01, R=0.1), "
                        f"seed {spec['seed']}, eps={eps}, theta={args.theta}, FP32 in/out",
            "n": n, "theta": args.theta, "eps": eps,
            "interactions_per_step": inter, "particle_terms_per_step": n_pp,
            "forces_per_s": n / (ms_step * 1e-3),
            "build_ms": build_ms, "walk_ms": walk_avg,
            "walk_interactions_per_s": inter / (walk_avg * 1e-3),
            "rms_rel_force_err": rms, "accuracy_targets": None if rms is None else args.samples,
            "n_nodes": tstats["n_nodes"],
            "quadrupole": quad,
            "learned_theta": learned,
            "launch": {"waves_per_block": args.waves_per_block, "xcd_chunk": args.xcd_chunk,
                       "target_order": args.target_order, "lds_share": args.lds_share,
                       "persistent": args.persistent, "targets_per_lane": args.targets_per_lane},
        },
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS,
            "traffic": measured_traffic(args.workload, args.theta),
            "kernel": "bh::k_walk<false, 1, 0, true, false>", "flops_per_unit": FLOPS_PER_INTERACTION,
            "units_per_launch": inter,
            "peak_note": "FP64 and unpacked FP32 vector rate; packed FP32 peak 157.3 TFLOP/s",
            "frac_of_packed_fp32_peak": achieved / PEAK_PACKED_FP32_TFLOPS,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        cb = cpu_baseline(pos32, mass32, args.theta, eps, spec["seed"], args.cpu_sample, args.cpu_sample_1t)
        line["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "one_thread")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
