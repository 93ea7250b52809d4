"""Benchmark of the sampled-silhouette hot path on one MI355X.

One step = one silhouette request end to end on the GPU: cluster index,
Phase 1 (PPS sampling, float64), sample packing, Phase 2 (weighted sums,
a_hat, b_hat, s_hat) and the float64 global mean, on the workload
n = 1e6, d = 32, k = 16 Gaussian blobs with Zipf(1.1) sizes, t = 256
samples per cluster, Euclidean distance.  The timed precision is bf16 MFMA
(float32 accumulation); the same steps in float32 give |delta s_mean|.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--metric eucl] [--prec bf16]

Prints one JSON line.  `value` is weighted distance evaluations per second of
the whole step: (n*S + sum_j |C_j| |F0_j|) / step time, with the inputs
resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X figures: published peaks, and unit-count derivations from them
# (256 CUs at 2.4 GHz).  157.3 TFLOP/s fp32 vector = 128 fp32 lanes / clk / CU
# doing packed FMAs (64 without packing); transcendental instructions
# (v_sqrt_f32) run at 32 lanes / clk / CU.
CU, CLK = 256, 2.4e9
PEAK = {
    "hbm_gbs": 8000.0,
    "fp32_vec_tflops": 157.3,
    "bf16_mfma_tflops": 2500.0,
    "fp8_mfma_tflops": 5000.0,
    "fp32_mfma_tflops": 157.3,
    "sqrt_tops": CU * 32 * CLK / 1e12,   # 19.66 T square roots / s
}
WORKLOAD = dict(n=1_000_000, d=32, k=16, t=256, seed=1)

# HBM bytes per Phase-2 launch on this workload from the two rocprofv3 PMC
# runs (FETCH_SIZE, WRITE_SIZE; scaled by a 256 MiB copy), valid only for the
# kernel source they were taken with (sha256 prefix of the source file).
TRAFFIC = {
    ("eucl", "bf16"): {"src": "paper_2607_01993_amd/csrc/k_phase2_mfma.hip", "sha256": "9991418b0ee7ddce",
                       "bytes": (136.7 + 12.3) * 1e6,
                       "profile": "profiles/hbm_traffic_zipf_n1e6_d32_k16_t256.md"},
}


def traffic_for(metric, prec):
    import hashlib
    rec = TRAFFIC.get((metric, prec))
    if rec is None:
        return None
    with open(os.path.join(ROOT, rec["src"]), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return rec["bytes"] if sha == rec["sha256"] else None


def phase2_roofline(metric, prec, d, n, S, kern_s):
    """Roofline of the Phase-2 launch: algorithmic work per launch (n*S pairs
    times the per-pair figure) over the average launch duration."""
    pairs = float(n) * S
    if metric == "eucl" and prec == "bf16":
        # two ceilings: the square root per pair (transcendental rate) and
        # the MFMA contraction (2d flops per pair); the nearer one governs
        # (the square root at d = 32, the matrix cores at d = 256), the
        # other is reported beside it
        sq = pairs / kern_s / 1e12
        mf = 2 * d * pairs / kern_s / 1e12
        sqrt_roof = {"bound": "alu", "achieved": sq, "peak": PEAK["sqrt_tops"], "unit": "TFLOP/s",
                     "frac": sq / PEAK["sqrt_tops"], "work": "1 square root per pair (counted as 1 flop)"}
        mfma_roof = {"bound": "mfma", "achieved": mf, "peak": PEAK["bf16_mfma_tflops"], "unit": "TFLOP/s",
                     "frac": mf / PEAK["bf16_mfma_tflops"], "work": f"2d = {2 * d} MFMA flops per pair"}
        if sqrt_roof["frac"] >= mfma_roof["frac"]:
            sqrt_roof["mfma"] = {x: mfma_roof[x] for x in ("achieved", "peak", "unit", "frac")}
            return sqrt_roof
        mfma_roof["sqrt"] = {x: sqrt_roof[x] for x in ("achieved", "peak", "unit", "frac")}
        return mfma_roof
    if metric in ("eucl", "cos") and prec in ("fp32", "bf16", "fp8"):
        pk = {"fp32": PEAK["fp32_mfma_tflops"], "bf16": PEAK["bf16_mfma_tflops"], "fp8": PEAK["fp8_mfma_tflops"]}[prec]
        ach = 2 * d * pairs / kern_s / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk,
                "work": f"2d = {2 * d} MFMA flops per pair"}
    # vector-ALU metrics: per pair and coordinate sub + add (Manhattan) or
    # sub, add, max, reciprocal, fma (Canberra); plus the weight fma
    per = {"manh": 2 * d + 2, "canb": 6 * d + 2, "eucl": 3 * d + 3, "cos": 3 * d + 4}[metric]
    ach = per * pairs / kern_s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK["fp32_vec_tflops"], "unit": "TFLOP/s",
            "frac": ach / PEAK["fp32_vec_tflops"], "work": f"{per} flops per pair"}


def _oracle_rows(args):
    import oracle
    X, L, k, metric, smp, rows = _CPU_STATE["job"]
    return oracle.estimate(X, L, k, metric, smp, rows=rows[args[0]:args[1]])["s"].shape[0]


_CPU_STATE = {}


def cpu_baseline(X, L, k, metric, t, seed, n_rows=16384, procs=None):
    """The float64 oracle, as it stands, on a bounded sample of the same
    workload: Phase 1 on all rows (one process), Phase 2 on n_rows seeded
    rows, extrapolated to all n rows (rows are independent in Phase 2).
    Phase 2 is timed twice: in one process, and split over `procs` forked
    processes (the host's cores, at most 16).  Runs before the GPU is
    touched, so forking is safe."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    n = X.shape[0]
    procs = procs or min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    smp = oracle.sample(X, L, k, metric, t, 0.01, seed, "pps")
    t1 = time.perf_counter()
    rows = np.sort(np.random.default_rng(123).choice(n, n_rows, replace=False))
    oracle.estimate(X, L, k, metric, smp, rows=rows)
    t2 = time.perf_counter()
    _CPU_STATE["job"] = (X, L, k, metric, smp, rows)
    step = (n_rows + procs - 1) // procs
    with mp.get_context("fork").Pool(procs) as pool:
        t3 = time.perf_counter()
        pool.map(_oracle_rows, [(a, min(n_rows, a + step)) for a in range(0, n_rows, step)])
        t4 = time.perf_counter()
    S = sum(f.shape[0] for f in smp["F"])
    p1 = sum(int(m.shape[0]) * int(f.shape[0]) for m, f in zip(smp["members"], smp["F0"]))
    one = (t1 - t0) + (t2 - t1) * n / n_rows
    many = (t1 - t0) + (t4 - t3) * n / n_rows
    return {
        "value": (n * S + p1) / many,
        "unit": "weighted dist evals/s",
        "cores": procs,
        "kind": "oracle",
        "sample": f"Phase 1 on all n={n} rows (one process, {t1 - t0:.1f} s) + Phase 2 on {n_rows} seeded rows "
                  f"over {procs} forked processes ({t4 - t3:.2f} s), Phase 2 time scaled by n/{n_rows}; NumPy "
                  f"float64 (host reports {os.cpu_count()} cores)",
        "one_thread": {"value": (n * S + p1) / one, "cores": 1,
                       "sample": f"same, Phase 2 in one process ({t2 - t1:.1f} s)"},
    }


def golden_mean(X, L, workload, metric):
    """The float64 oracle's full-size Eq. 9 mean stored in
    tests/golden/fullsize_means.json (written from oracle/ only), if it was
    computed from these very arrays; else None."""
    import hashlib
    path = os.path.join(ROOT, "tests", "golden", "fullsize_means.json")
    try:
        with open(path) as f:
            cases = json.load(f)["cases"]
    except OSError:
        return None
    h = hashlib.sha256()
    h.update(X.tobytes())
    h.update(L.tobytes())
    for c in cases:
        if c["workload"] == workload and c["metric"] == metric and c["data_sha256"] == h.hexdigest():
            return c["mean"]
    return None


def run_steps(native, Xd, Ld, k, metric, prec, t, seed, steps, warmup, out_a, out_b, out_s):
    """Warm-up, then `steps` timed requests; per-kernel event times."""
    import torch
    stats = {}
    info = {}

    def step(prof):
        ctx = native.silh_sample_init(Xd, Ld, k, metric, prec, "pps", t=t, delta=0.01, seed=seed,
                                      use_torch_alloc=False)
        if prof:
            native.silh_prof_enable(ctx, prof)
        S, _ = native.silh_pps_sample(ctx)
        res = native.silh_scores(ctx, a=True, b=True, s=True, mean=True)
        if prof:
            for name, (cnt, ms) in native.silh_prof_get(ctx).items():
                c0, m0 = stats.get(name, (0, 0.0))
                stats[name] = (c0 + cnt, m0 + ms)
        if "f0_offsets" not in info:
            info.update(native.silh_sample_view(ctx))
        native.silh_destroy(ctx)
        return S, res["mean"]

    for _ in range(warmup):
        step(False)
    # per-kernel breakdown from untimed steps (events around every kernel)
    for _ in range(max(2, steps // 4)):
        step(1)
    kstats = dict(stats)
    stats.clear()
    torch.cuda.synchronize()
    times = []
    t_all0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        S, mean = step(2)   # timed: events around the Phase-2 launch only
        times.append(time.perf_counter() - ts)
        print(f"# {metric}/{prec} step {i}: {times[-1] * 1e3:.3f} ms S={S} mean={mean:.7f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t_all0
    return {"S": S, "mean": mean, "t_all": t_all, "times": times, "stats": stats, "kstats": kstats, "info": info}


def run_rows(native, torch, Xd, Ld, k, metric, prec, t, seed, steps, full_mean, eps=0.01, delta=0.01):
    """gl-pps-s (Eq. 10): Phase 1 as in a full request, then Phase 2 only for
    m = ceil((2/eps^2) ln(2/delta)) uniform row draws."""
    n = Xd.shape[0]
    m = native.silh_rows_for(eps, delta)
    times, mean, S = [], None, 0
    for i in range(steps + 1):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ctx = native.silh_sample_init(Xd, Ld, k, metric, prec, "pps", t=t, delta=0.01, seed=seed,
                                      use_torch_alloc=False)
        S, _ = native.silh_pps_sample(ctx)
        rows = native.silh_draw_rows(seed + 1000, n, m)
        mean = native.silh_scores_rows(ctx, rows, a=False, b=False, s=False, mean=True)["mean"]
        native.silh_destroy(ctx)
        if i > 0:   # the first request is a warm-up
            times.append(time.perf_counter() - ts)
    t_req = sum(times) / len(times)
    return {"m": m, "eps2": eps, "delta2": delta, "ms_per_request": t_req * 1e3,
            "phase2_pairs": m * S, "s_bar": mean, "abs_delta_vs_s_hat_2": abs(mean - full_mean)}


def run_graph(native, Xd, Ld, k, metric, prec, t, seed, steps, warmup, work, eager_mean):
    """The same request captured once into a HIP graph (include/silh_graph.h)
    and replayed: every step recomputes the index, Phase 1, packing, Phase 2
    and the mean from X and the labels, with no host round trip in between."""
    t0 = time.perf_counter()
    g = native.SweepGraph(Xd, Ld.view(1, -1), [k], metric, prec, t=t, seed=seed, chains=1)
    capture = time.perf_counter() - t0
    for _ in range(warmup):
        g.run()
    times = []
    res = None
    for _ in range(steps):
        t0 = time.perf_counter()
        res = g.run()
        times.append(time.perf_counter() - t0)
    info = g.info()
    g.close()
    tm = sum(times) / len(times)
    return {"value": work / tm, "ms_per_step": tm * 1e3, "capture_ms": capture * 1e3, "nodes": info["nodes"],
            "s_mean": float(res["means"][0]), "same_mean_as_eager": bool(res["means"][0] == eager_mean),
            "note": "one request as a captured graph, replayed; each step synchronises once and reads "
                    "the mean back"}


def run_leg(native, Xd, Ld, k, metric, prec, t, seed, steps, a, b, s, work_fn=None, gold=None):
    """A request workload other than the headline: steps requests (one
    warm-up), step time, Phase-2 launch time, its roofline, |mean - oracle|."""
    import numpy as np
    r = run_steps(native, Xd, Ld, k, metric, prec, t, seed, steps, 1, a, b, s)
    c2, m2 = r["stats"].get("phase2", (0, 0.0))
    n, d = Xd.shape
    sizes = np.bincount(Ld.cpu().numpy(), minlength=k)
    p1 = int((sizes * np.diff(r["info"]["f0_offsets"])).sum())
    work = n * r["S"] + p1
    out = {"value": work / (r["t_all"] / steps), "ms_per_step": r["t_all"] / steps * 1e3,
           "phase2_ms": m2 / max(c2, 1), "S": r["S"], "s_mean": r["mean"],
           "phase2_roofline": phase2_roofline(metric, prec, d, n, r["S"], m2 / max(c2, 1) / 1e3)}
    if gold is not None:
        out["oracle_mean"] = gold
        out["abs_delta_vs_oracle"] = abs(r["mean"] - gold)
    return out


def run_serving(native, torch, requests=48, load=0.5):
    """A short serving run: the resident 32-dataset pool, `requests` requests
    queued at once (saturation), then the same mix as Poisson arrivals at
    load x saturation; p50/p99 latency overall and per metric.  Both server
    modes: Phase 2 of concurrent requests in shared launches ("batched") and
    each request's own launch on its worker stream ("own"), at the same
    arrival rate (load x the batched saturation)."""
    from paper_2607_01993_amd import serving
    specs, data, reqs = serving.build_workload(requests, torch.device("cuda:0"))
    out = {"requests": len(reqs),
           "note": "32 resident datasets (n 1e4..2e6, d 16/64/256, eucl/cos bf16, manh/canb fp32), Voronoi "
                   "requests k 2..128, t 64/256/1024"}
    rate = None
    for mode in ("batched", "own"):
        srv = native.Server(workers=4, hbm_budget_bytes=96 << 30, batched=mode == "batched")
        ids = [srv.add_dataset(X) for X in data]
        serving.run_closed(srv, ids, reqs)  # warm-up: block caches, and the autotuner's keys of every request
        res, secs = serving.run_closed(srv, ids, reqs)
        sat = len(reqs) / secs
        pairs = float(sum(specs[r["dataset"]]["n"] * x["S"] for r, x in zip(reqs, res)))
        if rate is None:
            rate = load * sat
        rr = serving.run_poisson(srv, ids, reqs, rate, seed=11)
        out[mode] = {"saturation_req_s": sat, "weighted_dist_evals_per_s_closed": pairs / secs, "rate_req_s": rate,
                     "latency_ms": serving.summarize(rr, reqs), "shared_launches": srv.launches()}
        srv.close()
        print(f"# serving [{mode}]: saturation {sat:.1f} req/s, p50 {out[mode]['latency_ms']['p50_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--metric", default="eucl")
    ap.add_argument("--prec", default="bf16")
    ap.add_argument("--compare-steps", type=int, default=5,
                    help="steps of the float32 comparison run and of the Manhattan run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the directional (n = 4e6, d = 128), d = 256 and serving legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 256 MiB once first (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the multi-GPU row "
              "sharding of the path is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_01993_amd import native, synth

    n, d, k, t, seed = (WORKLOAD[x] for x in ("n", "d", "k", "t", "seed"))
    X, L = synth.config_zipf_gauss(n=n, d=d, k=k, seed=seed)
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the oracle's Phase 2 runs in forked processes
        print("# timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(X, L, k, args.metric, t, seed)
    gold = golden_mean(X, L, "zipf-gauss-blobs", args.metric)
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(L).cuda()
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = torch.empty_like(a)
    native.load_library()
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# copy calibration: 268435456 bytes read, 268435456 bytes written", file=sys.stderr)
        del src, dst
    print(f"# workload ready: n={n} d={d} k={k} t={t}", file=sys.stderr, flush=True)

    main_run = run_steps(native, Xd, Ld, k, args.metric, args.prec, t, seed, args.steps, args.warmup,
                         a, b, s)
    S = main_run["S"]
    sizes = np.bincount(L, minlength=k)
    f0 = np.diff(main_run["info"]["f0_offsets"])
    p1 = int((sizes * f0).sum())
    work = n * S + p1
    t_step = main_run["t_all"] / args.steps
    stats = main_run["stats"]
    p2_cnt, p2_ms = stats.get("phase2", (0, 0.0))
    p2_s = p2_ms / max(p2_cnt, 1) / 1e3
    roof = phase2_roofline(args.metric, args.prec, d, n, S, p2_s)
    roof.update({"traffic": traffic_for(args.metric, args.prec), "kernel": "k_p2_mfma" if args.prec in ("bf16", "fp32") and
                 args.metric in ("eucl", "cos") else "k_p2_valu", "kernel_ms": p2_s * 1e3})

    compare = {}
    if args.compare_steps > 0 and args.metric == "eucl":
        ref_prec = "fp32" if args.prec != "fp32" else "bf16"
        r = run_steps(native, Xd, Ld, k, "eucl", ref_prec, t, seed, args.compare_steps, 1, a, b, s)
        c2, m2 = r["stats"].get("phase2", (0, 0.0))
        compare[f"eucl_{ref_prec}"] = {
            "value": work / (r["t_all"] / args.compare_steps), "ms_per_step": r["t_all"] / args.compare_steps * 1e3,
            "phase2_ms": m2 / max(c2, 1), "s_mean": r["mean"],
            "abs_delta_s_mean": abs(r["mean"] - main_run["mean"]),
            "abs_delta_vs_oracle": abs(r["mean"] - gold) if gold is not None else None}
        r = run_steps(native, Xd, Ld, k, "manh", "fp32", t, seed, args.compare_steps, 1, a, b, s)
        c2, m2 = r["stats"].get("phase2", (0, 0.0))
        sz = np.diff(r["info"]["f0_offsets"])
        w2 = n * r["S"] + int((sizes * sz).sum())
        compare["manh_fp32"] = {
            "value": w2 / (r["t_all"] / args.compare_steps), "ms_per_step": r["t_all"] / args.compare_steps * 1e3,
            "phase2_ms": m2 / max(c2, 1),
            "phase2_roofline": phase2_roofline("manh", "fp32", d, n, r["S"], m2 / max(c2, 1) / 1e3)}

    if args.compare_steps > 0 and not args.no_large:
        # the directional workload: n = 4e6, d = 128, k = 64 vMF blobs, t = 512, cosine
        print("# generating the directional workload (n = 4e6, d = 128)", file=sys.stderr, flush=True)
        Xv, Lv = synth.config_vmf_cos()
        gv = golden_mean(Xv, Lv, "vmf-blobs", "cos")
        Xvd, Lvd = torch.from_numpy(Xv).cuda(), torch.from_numpy(Lv).cuda()
        del Xv, Lv
        av = torch.empty(Xvd.shape[0], dtype=torch.float32, device="cuda")
        bv, sv = torch.empty_like(av), torch.empty_like(av)
        for prec, steps in (("bf16", args.compare_steps), ("fp8", args.compare_steps), ("fp32", 2)):
            compare[f"vmf_n4e6_d128_k64_t512_cos_{prec}"] = run_leg(native, Xvd, Lvd, 64, "cos", prec, 512, 2,
                                                                    steps, av, bv, sv, gold=gv)
        del Xvd, Lvd, av, bv, sv
        torch.cuda.empty_cache()
        # long rows: n = 5e5, d = 256, k = 16 Zipf Gaussian blobs, t = 256, Euclidean bf16
        Xw, Lw = synth.config_zipf_gauss(n=500_000, d=256, k=16, seed=4)
        Xwd, Lwd = torch.from_numpy(Xw).cuda(), torch.from_numpy(Lw).cuda()
        aw = torch.empty(Xwd.shape[0], dtype=torch.float32, device="cuda")
        bw, sw = torch.empty_like(aw), torch.empty_like(aw)
        compare["zipf_n5e5_d256_k16_t256_eucl_bf16"] = run_leg(native, Xwd, Lwd, 16, "eucl", "bf16", 256, 4,
                                                               args.compare_steps, aw, bw, sw)
        del Xwd, Lwd, aw, bw, sw
        torch.cuda.empty_cache()
        print("# serving leg", file=sys.stderr, flush=True)
        compare["serving"] = run_serving(native, torch)

    if args.compare_steps > 0:
        compare["graph_replay"] = run_graph(native, Xd, Ld, k, args.metric, args.prec, t, seed, args.steps,
                                            args.warmup, work, main_run["mean"])
        compare["gl_pps_s"] = run_rows(native, torch, Xd, Ld, k, args.metric, args.prec, t, seed,
                                       args.compare_steps, main_run["mean"])

    times_ms = np.array(main_run["times"]) * 1e3
    out = {
        "metric": "weighted dist evals/s",
        "value": work / t_step,
        "unit": "weighted dist evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8", "fp32_valu": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"zipf-gauss-blobs n={n} d={d} k={k} t={t} metric={args.metric} "
                               f"prec={args.prec} sampler=pps delta=0.01 seed={seed}",
                   "n": n, "d": d, "k": k, "t": t, "S": S, "phase1_dists": p1,
                   "parallelism": "single GPU"},
        "request_latency_ms": {"p50": float(np.percentile(times_ms, 50)),
                               "p99": float(np.percentile(times_ms, 99)),
                               "note": "one request = one whole step, issued back to back"},
        "phase2_pairs_per_s": n * S / p2_s,
        "kernel_avg_ms": {name: round(ms / max(cnt, 1), 4) for name, (cnt, ms) in sorted(main_run["kstats"].items())
                          if cnt},
        "kernel_avg_ms_note": "from untimed steps with events around every kernel; phase2 in the roofline is "
                              "from the timed steps",
        "roofline": roof,
        "s_mean": main_run["mean"],
        "oracle_mean": gold,
        "abs_delta_vs_oracle": abs(main_run["mean"] - gold) if gold is not None else None,
        "compare": compare,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
