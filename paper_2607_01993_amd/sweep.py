"""k-sweep measurement: the global silhouette of 256 clusterings of one
dataset (k = 2..257) and the k that maximises it (Section 5, selection of
the best value of k), through silh_sweep (worker streams) or, with
--graph, through one captured HIP graph (silh_graph_*: capture and
instantiation timed apart from the runs; the runs replay the graph).

    python -m paper_2607_01993_amd.sweep [--metric eucl] [--prec bf16] [--m 0] [--kmax 257] [--graph] [--out FILE]

Workload: n = 5e5 rows of d = 64 exponential blobs (16 blobs, offsets
U[0, 10]^64, x = offset + Exp(1) per coordinate, seed 3); clustering k is the
Voronoi partition of k rows drawn with seed (3, k) (Euclidean, ties to the
lowest index, computed on the device); t = 128, delta = 0.01.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def build(n=500_000, d=64, kmin=2, kmax=257, seed=3):
    import torch

    from . import synth
    X = torch.from_numpy(synth.config_sweep(n=n, d=d, seed=seed)).cuda()
    ks = list(range(kmin, kmax + 1))
    L = torch.empty((len(ks), n), dtype=torch.int32, device="cuda")
    for i, k in enumerate(ks):
        L[i] = synth.voronoi_labels_device(X, synth.voronoi_centers(n, k, (seed, k)))
    torch.cuda.synchronize()
    return X, L, ks


def run(X, L, ks, metric, prec, t=128, m=0, workers=4, seed=3, reps=1):
    import torch

    from . import native
    res = None
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = native.silh_sweep(X, L, ks, metric, prec, t=t, seed=seed, m=m, workers=workers)
        times.append(time.perf_counter() - t0)
    return res, min(times)


def run_graph(X, L, ks, metric, prec, t=128, chains=4, seed=3, reps=2):
    """Capture once, then `reps` runs; returns the last result, the capture
    time and the fastest run (each run includes the host read-back)."""
    import torch

    from . import native
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = native.SweepGraph(X, L, ks, metric, prec, t=t, seed=seed, chains=chains)
    create = time.perf_counter() - t0
    info = g.info()
    times, res = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        res = g.run()
        times.append(time.perf_counter() - t0)
    g.close()
    return res, create, min(times), times, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--metric", default="eucl")
    ap.add_argument("--prec", default="bf16")
    ap.add_argument("--m", type=int, default=0)
    ap.add_argument("--kmax", type=int, default=257)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--graph", action="store_true", help="one captured HIP graph instead of worker streams")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    X, L, ks = build(kmax=args.kmax)
    log(f"{len(ks)} clusterings ready (n={X.shape[0]}, d={X.shape[1]})")
    extra = {}
    if args.graph:
        if args.m:
            raise SystemExit("--graph runs the full Phase 2 (m = 0)")
        res, create, secs, times, info = run_graph(X, L, ks, args.metric, args.prec, chains=args.workers,
                                                   reps=args.reps)
        extra = {"mode": "graph", "chains": args.workers, "capture_s": create, "run_s": times,
                 "graph": info, "reruns": res["reruns"]}
    else:
        res, secs = run(X, L, ks, args.metric, args.prec, m=args.m, workers=args.workers, reps=args.reps)
        extra = {"mode": "workers", "workers": args.workers}
    means = res["means"]
    out = {
        "workload": f"k-sweep: exp blobs n={X.shape[0]} d={X.shape[1]}, Voronoi k={ks[0]}..{ks[-1]}, t=128, "
                    f"delta 0.01, metric={args.metric} prec={args.prec} m={args.m}",
        "clusterings": len(ks), "seconds": secs, "clusterings_per_s": len(ks) / secs,
        "best_k": ks[res["best"]], "best_mean": float(means[res["best"]]),
        "means_head": [float(v) for v in means[:8]], **extra,
    }
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(json.dumps(out) + "\n")


if __name__ == "__main__":
    main()
