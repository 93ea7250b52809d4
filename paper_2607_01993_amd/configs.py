"""Phase-2 measurements on each workload shape, with the roofline that bounds
each path.

    python -m paper_2607_01993_amd.configs [--out FILE] [--only zipf,d256] [--metrics canb,manh]

Workloads (seeded, synthetic):
  small       n = 2,000, d = 8, k = 4 Gaussian blobs, t = 64
  zipf        n = 1e6, d = 32, k = 16 Zipf Gaussian blobs, t = 256
  directional n = 4e6, d = 128, k = 64 vMF blobs (kappa 50), t = 512, cosine
  sweep-k64   n = 5e5, d = 64 exponential blobs, Voronoi k = 64, t = 128
  d256        n = 5e5, d = 256, k = 16 Zipf Gaussian blobs, t = 256

For every (workload, metric, operands) the Phase-2 launch is timed with HIP
events (median of 5 requests after one warm-up) and reported as pairs/s,
MFMA TFLOP/s (2d flops per pair) against the operand type's peak, and for
Euclidean the square-root rate against its 19.66e12/s ceiling; vector-ALU
metrics against 157.3 TFLOP/s.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys

PEAK_MFMA = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
SQRT_PEAK = 19.6608  # 1e12 square roots / s
VALU_PEAK = 157.3
VALU_FLOPS = {"manh": lambda d: 2 * d + 2, "canb": lambda d: 6 * d + 2, "eucl": lambda d: 3 * d + 3,
              "cos": lambda d: 3 * d + 4}


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def measure(native, X, L, k, metric, prec, t, reps=5):
    times, S = [], 0
    for i in range(reps + 1):
        ctx = native.silh_sample_init(X, L, k, metric, prec, "pps", t=t, seed=1)
        native.silh_prof_enable(ctx, 2)
        S, _ = native.silh_pps_sample(ctx)
        native.silh_scores(ctx, a=False, b=False, s=False, mean=True)
        ms = native.silh_prof_get(ctx)["phase2"][1]
        native.silh_destroy(ctx)
        if i > 0:
            times.append(ms)
    ms = statistics.median(times)
    n, d = X.shape
    pairs = float(n) * S / (ms * 1e-3)
    out = {"metric": metric, "prec": prec, "n": n, "d": d, "k": k, "t": t, "S": S, "phase2_ms": ms,
           "pairs_per_s": pairs}
    mfma = metric in ("eucl", "cos") and prec in PEAK_MFMA and not (prec == "fp32" and d > 128)
    if mfma:
        tf = 2 * d * pairs / 1e12
        out["mfma_tflops"] = tf
        out["mfma_frac"] = tf / PEAK_MFMA[prec]
        if metric == "eucl":
            out["sqrt_frac"] = pairs / 1e12 / SQRT_PEAK
    else:
        tf = VALU_FLOPS[metric](d) * pairs / 1e12
        out["valu_tflops"] = tf
        out["valu_frac"] = tf / VALU_PEAK
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--skip-directional", action="store_true")
    ap.add_argument("--only", default=None, help="comma-separated workloads (small, zipf, sweep-k64, d256, directional)")
    ap.add_argument("--metrics", default=None, help="comma-separated metrics to measure (default: all)")
    args = ap.parse_args()
    only = set(args.only.split(",")) if args.only else None
    mets = set(args.metrics.split(",")) if args.metrics else None

    def want(workload, metric=None):
        return (only is None or workload in only) and (metric is None or mets is None or metric in mets)
    import torch

    from . import native, synth

    def dev(X, L):
        return torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda()

    rows = []
    if want("small"):
        X, L = dev(*synth.config_small())
        for metric, prec in (("eucl", "fp32"), ("eucl", "bf16")):
            if want("small", metric):
                rows.append({"workload": "small", **measure(native, X, L, 4, metric, prec, 64)})
    if want("zipf"):
        X, L = dev(*synth.config_zipf_gauss())
        for metric, prec in (("eucl", "bf16"), ("eucl", "fp32"), ("cos", "bf16"), ("manh", "fp32"), ("canb", "fp32")):
            if want("zipf", metric):
                rows.append({"workload": "zipf", **measure(native, X, L, 16, metric, prec, 256)})
        log("zipf done")
        del X, L
    if want("sweep-k64"):
        Xe = synth.config_sweep()
        cen = synth.voronoi_centers(Xe.shape[0], 64, (3, 64))
        Le = synth.voronoi_labels(Xe, cen)
        X, L = dev(Xe, Le)
        for metric, prec in (("eucl", "bf16"), ("canb", "fp32")):
            if want("sweep-k64", metric):
                rows.append({"workload": "sweep-k64", **measure(native, X, L, 64, metric, prec, 128)})
        log("sweep-k64 done")
    if want("d256"):
        n = 500_000
        Xg, Lg = synth.gaussian_blobs(n, 256, 16, seed=9, sizes=synth.zipf_sizes(n, 16), sigma=(0.5, 2.0))
        X, L = dev(Xg, Lg)
        for metric, prec in (("eucl", "bf16"), ("cos", "fp8"), ("manh", "fp32")):
            if want("d256", metric):
                rows.append({"workload": "d256", **measure(native, X, L, 16, metric, prec, 256, reps=3)})
        log("d256 done")
        del X, L
    if not args.skip_directional and want("directional", "cos"):
        Xv, Lv = synth.config_vmf_cos()
        log("directional data ready")
        X, L = dev(Xv, Lv)
        del Xv, Lv
        for prec in ("bf16", "fp8", "fp32"):
            rows.append({"workload": "directional", **measure(native, X, L, 64, "cos", prec, 512, reps=3)})
            log(f"directional {prec} done")
    line = json.dumps({"phase2_by_workload": rows})
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
