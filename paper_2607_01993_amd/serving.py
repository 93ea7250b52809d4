"""Serving measurement: silhouette requests against a pool of resident
datasets, with Poisson arrivals, through the library's serving runtime
(include/silh_server.h).

    python -m paper_2607_01993_amd.serving [--requests R] [--workers W] [--mode batched|own|both] [--out FILE]

Workload: 32 resident datasets (n log-uniform in [1e4, 2e6], d in {16, 64,
256}, one metric each: Euclidean and cosine in bf16 MFMA, Manhattan and
Canberra in float32), requests with k ~ U{2..128} (Voronoi clusterings), t
in {64, 256, 1024}, delta = 0.01.  First a closed run (every request queued at
once) gives the saturation rate; then for each load factor f the same request
mix arrives as a Poisson process of rate f * saturation, and the per-request
latency (completion minus arrival) is reported as p50 / p99, overall and per
metric.  Mode "batched" runs the Phase 2 of concurrent requests in shared
launches over (request, row-block) work items; "own" gives every request its
own Phase-2 launch on its worker stream.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


PRECS = {"eucl": "bf16", "cos": "bf16", "manh": "fp32", "canb": "fp32"}


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def build_workload(requests, device, pool_seed=5, req_seed=7):
    import torch

    from . import synth
    specs = synth.serving_pool_specs(seed=pool_seed)
    data = [synth.serving_dataset(s, device) for s in specs]
    torch.cuda.synchronize()
    log(f"pool ready: {len(specs)} datasets, {sum(s['n'] for s in specs)} rows")
    reqs = synth.serving_requests(specs, requests, seed=req_seed)
    for r in reqs:
        X = data[r["dataset"]]
        cen = synth.voronoi_centers(X.shape[0], r["k"], r["centers_seed"])
        r["labels"] = synth.voronoi_labels_device(X, cen)
        spec = specs[r["dataset"]]
        r["metric"] = spec["metric"]
        r["prec"] = PRECS[spec["metric"]]
        r["pairs_est"] = None
    torch.cuda.synchronize()
    log(f"{len(reqs)} requests with Voronoi labels ready")
    return specs, data, reqs


def run_closed(srv, ids, reqs):
    t0 = srv.now_ns()
    tks = [srv.submit(ids[r["dataset"]], r["labels"], r["k"], r["metric"], r["prec"], t=r["t"], seed=r["seed"])
           for r in reqs]
    res = [srv.wait(tk) for tk in tks]
    t1 = max(x["done_ns"] for x in res)
    return res, (t1 - t0) / 1e9


def run_poisson(srv, ids, reqs, rate, seed):
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(reqs))
    start = srv.now_ns() + 20_000_000
    arrivals = start + (np.cumsum(gaps) * 1e9).astype(np.int64)
    tks = []
    last_print = time.time()
    for r, at in zip(reqs, arrivals):
        while True:
            now = srv.now_ns()
            if now >= at:
                break
            wait = (at - now) / 1e9
            if wait > 0.002:
                time.sleep(wait - 0.001)
        tks.append((srv.submit(ids[r["dataset"]], r["labels"], r["k"], r["metric"], r["prec"], t=r["t"],
                               seed=r["seed"]), int(at)))
        if time.time() - last_print > 30:
            log(f"  submitted {len(tks)}/{len(reqs)}")
            last_print = time.time()
    res = []
    for tk, at in tks:
        x = srv.wait(tk)
        x["arrival_ns"] = at
        res.append(x)
    return res


def summarize(res, reqs=None, key_from="submit_ns"):
    lat = np.array([(x["done_ns"] - x[key_from]) / 1e6 for x in res])
    queue = np.array([(x["start_ns"] - x["submit_ns"]) / 1e6 for x in res])
    out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "queue_p50_ms": float(np.percentile(queue, 50)),
           "failed": int(sum(x["status"] != "SILH_OK" for x in res))}
    if reqs is not None:
        by = {}
        for m in ("eucl", "cos", "manh", "canb"):
            v = np.array([lt for lt, r in zip(lat, reqs) if r["metric"] == m])
            if v.size:
                by[m] = {"n": int(v.size), "p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99))}
        out["by_metric"] = by
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=96)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=96.0)
    ap.add_argument("--loads", default="0.25,0.5,0.75,0.9")
    ap.add_argument("--mode", default="both", choices=["batched", "own", "both"])
    ap.add_argument("--rate", type=float, default=0.0,
                    help="arrival rate (req/s) of every load point, as multiples of it; 0: of the batched saturation")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    import torch

    from . import native
    dev = torch.device("cuda:0")
    specs, data, reqs = build_workload(args.requests, dev)
    modes = ["batched", "own"] if args.mode == "both" else [args.mode]
    runs = {}
    base_rate = args.rate
    for mode in modes:
        srv = native.Server(workers=args.workers, hbm_budget_bytes=int(args.budget_gib * (1 << 30)),
                            batched=mode == "batched")
        ids = [srv.add_dataset(X) for X in data]
        # warm-up: one request of each metric
        seen = set()
        warm = []
        for r in reqs:
            if r["metric"] not in seen:
                seen.add(r["metric"])
                warm.append(r)
        run_closed(srv, ids, warm)
        log(f"[{mode}] warm-up done")
        res, secs = run_closed(srv, ids, reqs)
        sat = len(reqs) / secs
        closed = summarize(res, reqs)
        log(f"[{mode}] closed run: {len(reqs)} requests in {secs:.2f} s -> saturation {sat:.2f} req/s; {closed}")
        pairs = float(sum(specs[r["dataset"]]["n"] * x["S"] for r, x in zip(reqs, res)))
        if base_rate <= 0.0:
            base_rate = sat  # the load points of every mode are fractions of the first mode's saturation
        loads = []
        for i, f in enumerate(float(v) for v in args.loads.split(",")):
            rr = run_poisson(srv, ids, reqs, f * base_rate, seed=11 + i)
            s = summarize(rr, reqs)
            s.update({"load": f, "rate_req_s": f * base_rate})
            loads.append(s)
            log(f"[{mode}] load {f}: {s}")
        runs[mode] = {"saturation_req_s": sat, "closed_run": closed, "weighted_dist_evals_per_s_closed": pairs / secs,
                      "loads": loads, "shared_launches": srv.launches()}
        srv.close()
    out = {
        "workload": "serving pool: 32 datasets n~10^U[4,log10 2e6], d in {16,64,256}, metric per dataset "
                    "(eucl/cos bf16 MFMA, manh/canb fp32), k~U{2..128} Voronoi, t in {64,256,1024}, delta 0.01",
        "requests": len(reqs), "workers": args.workers, "rate_base_req_s": base_rate, "modes": runs,
        "metric_mix": {m: sum(1 for r in reqs if r["metric"] == m) for m in ("eucl", "cos", "manh", "canb")},
    }
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
