"""Write tests/golden/fullsize_means.json: the float64 oracle's value of the
global estimate s_hat_2 (Eq. 9, the mean of s_hat over all n elements after
Phase 1 and Phase 2 of Algorithm 1) at full size, for

  * the Zipf Gaussian-blob workload (n = 1e6, d = 32, k = 16, t = 256,
    delta = 0.01, Philox key 1), Euclidean and Manhattan;
  * the directional workload (n = 4e6, d = 128, k = 64 vMF blobs, t = 512,
    delta = 0.01, Philox key 2), cosine.

Only the oracle computes: `oracle.sample` (Phase 1), `oracle.estimate` (Phase
2, pair by pair; row chunks in worker processes) for the Gaussian blobs, and
`oracle.cosine_estimate` (the same sums by the cosine distance's linear form)
for the directional workload.  Inputs come from the seeded generators; a
SHA-256 of X and labels is stored so a test can tell that it regenerated the
same data.

    python tests/golden/make_fullsize.py [--procs 8]

Takes about ten minutes on 8 cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2607_01993_amd import synth  # noqa: E402  (seeded inputs only)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_means.json")

_G = {}


def data_hash(X, L) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X).tobytes())
    h.update(np.ascontiguousarray(L).tobytes())
    return h.hexdigest()


def _chunk(args):
    r0, r1 = args
    X, L, k, metric, smp = _G["X"], _G["L"], _G["k"], _G["metric"], _G["smp"]
    est = oracle.estimate(X, L, k, metric, smp, rows=np.arange(r0, r1))
    return r0, est["s"]


def pairwise_mean(X, L, k, metric, smp, procs):
    _G.update(X=X, L=L, k=k, metric=metric, smp=smp)
    n = X.shape[0]
    step = 8192
    s = np.empty(n)
    with get_context("fork").Pool(procs) as pool:
        for r0, part in pool.imap_unordered(_chunk, [(a, min(n, a + step)) for a in range(0, n, step)]):
            s[r0:r0 + part.shape[0]] = part
    return oracle.global_mean(s)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    out = {"note": "float64 oracle values of the Eq. 9 mean at full size; written by make_fullsize.py",
           "cases": []}
    X, L = synth.config_zipf_gauss()
    h = data_hash(X, L)
    for metric in ("eucl", "manh"):
        t0 = time.time()
        smp = oracle.sample(X, L, 16, metric, 256, 0.01, 1)
        mean = pairwise_mean(X, L, 16, metric, smp, args.procs)
        S = int(sum(f.shape[0] for f in smp["F"]))
        print(f"zipf {metric}: S={S} mean={mean!r} ({time.time() - t0:.0f} s)", flush=True)
        out["cases"].append({"workload": "zipf-gauss-blobs", "n": 1_000_000, "d": 32, "k": 16, "t": 256,
                             "delta": 0.01, "seed": 1, "sampler": "pps", "metric": metric, "S": S,
                             "mean": mean, "data_sha256": h})
    del X, L
    X, L = synth.config_vmf_cos()
    h = data_hash(X, L)
    t0 = time.time()
    smp = oracle.sample(X, L, 64, "cos", 512, 0.01, 2)
    est = oracle.cosine_estimate(X, L, 64, smp)
    S = int(sum(f.shape[0] for f in smp["F"]))
    print(f"vmf cos: S={S} mean={est['mean']!r} ({time.time() - t0:.0f} s)", flush=True)
    out["cases"].append({"workload": "vmf-blobs", "n": 4_000_000, "d": 128, "k": 64, "t": 512,
                         "delta": 0.01, "seed": 2, "sampler": "pps", "metric": "cos", "S": S,
                         "mean": est["mean"], "data_sha256": h})
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
