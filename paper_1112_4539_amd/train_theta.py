"""Trains the opening-parameter network shipped as weights/theta_clumpy4m.json.

Recipe (run on the GPU: ``python -m paper_1112_4539_amd.train_theta``): 32 clumpy fields of
4,194,304 particles (the field recipe of the headline workload, seeds 300-331, eps 1e-4; the
headline field itself, seed 2, is not among them), 4096 sampled walk groups of each labelled
with the cost-optimal allocation at RMS 1e-3 (learn.label_sampled), then 80 epochs of Adam on
batches of 1024 (learn.train).  Labels, features and training all run in the library's kernels;
the result is deterministic for a given library build up to the order of floating-point
reductions on the GPU.
"""
import argparse
import os
import sys
import time

import torch

from paper_1112_4539_amd import learn


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=4194304)
    ap.add_argument("--seeds", type=int, nargs=2, default=(300, 332), metavar=("FIRST", "END"))
    ap.add_argument("--groups", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=80)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--out", default=learn.DEFAULT_WEIGHTS)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    X, L = learn.build_dataset_sampled(range(*a.seeds), a.n, a.groups, log=log)
    t1 = time.perf_counter()
    net, hist = learn.train(X, L, epochs=a.epochs, batch=a.batch, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"fields": f"clumpy, n={a.n}, seeds {a.seeds[0]}-{a.seeds[1] - 1}, eps 1e-4",
            "sampled_groups_per_field": a.groups, "rows": int(L.shape[0]), "epochs": a.epochs, "batch": a.batch,
            "label_target_rms": learn.TARGET, "theta_grid": list(learn.THETA_GRID),
            "loss_first_last": [hist[0], hist[-1]], "label_s": round(t1 - t0, 1), "train_s": round(t2 - t1, 1)}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    learn.save_net(a.out, net, info)
    log(f"[train_theta] {a.out}: {info}")


if __name__ == "__main__":
    main()
