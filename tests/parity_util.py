"""Shared bars and helpers of the GPU parity tests (HIP path against the
float64 oracle).

Bars: sample index sets bit-exact (a decision may differ only where the
uniform lies within 1e-12 of the oracle's rate: both sides decide in float64
but sum W(e_bar) in different orders); float32 a_hat, b_hat within 1e-5
relative; s_hat and the mean within 4e-5 absolute (Lemma 2 with rho = 1e-5:
4 rho / (1 - rho))."""
import hashlib
import json
import os

import numpy as np
import torch

import oracle

A_B_RTOL = 1e-5
S_ATOL = 4.0e-5
# bf16 operands (float32 accumulation): per-element and mean bars
LOWP_S_ATOL = 1e-2
LOWP_MEAN_ATOL = 1e-3
# fp8 (e4m3) operands: the same bars as bf16
FP8_S_ATOL = LOWP_S_ATOL


def dev(X, L):
    return torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda()


def assert_same_sets(smp_o, view, X_n, seed, sampler, t):
    """Sample sets equal cluster by cluster, up to float64 decision ties."""
    k = len(smp_o["F"])
    assert view["S"] == sum(f.shape[0] for f in smp_o["F"])
    stream = oracle.STREAM_PPS if sampler == "pps" else oracle.STREAM_UNI
    for j in range(k):
        g = view["gid"][view["offsets"][j]:view["offsets"][j + 1]]
        o = smp_o["F"][j]
        if not np.array_equal(g, o):
            diff = np.setxor1d(g, o)
            u = oracle.uniform53(seed, diff.astype(np.uint64), stream)
            margin = np.abs(u - smp_o["p"][diff])
            assert np.all(margin < 1e-12), (j, diff[:10], margin[:10])


def compare_scores(gpu, ref, rows=None, prec="fp32"):
    a = gpu["a"].cpu().numpy().astype(np.float64)
    b = gpu["b"].cpu().numpy().astype(np.float64)
    s = gpu["s"].cpu().numpy().astype(np.float64)
    if rows is not None:
        a, b, s = a[rows], b[rows], s[rows]
    if prec in ("fp32", "fp32_valu"):
        np.testing.assert_allclose(a, ref["a"], rtol=A_B_RTOL, atol=1e-30)
        np.testing.assert_allclose(b, ref["b"], rtol=A_B_RTOL, atol=1e-30)
        assert np.max(np.abs(s - ref["s"])) <= S_ATOL
    else:
        bar = FP8_S_ATOL if prec == "fp8" else LOWP_S_ATOL
        err = np.abs(s - ref["s"])
        print(f"{prec}: max|ds|={err.max():.3e} mean|ds|={err.mean():.3e}")
        assert err.max() <= bar, err.max()
    assert np.all(np.abs(s) <= 1.0)


def mean_tol(prec):
    return S_ATOL if prec in ("fp32", "fp32_valu") else LOWP_MEAN_ATOL




GOLDEN_FULLSIZE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_means.json")


def golden_mean(X, L, workload, metric):
    """The float64 oracle's Eq. 9 mean at full size for this workload and
    metric (tests/golden/make_fullsize.py), after checking that X and the
    labels are the arrays it was computed from."""
    with open(GOLDEN_FULLSIZE) as f:
        cases = json.load(f)["cases"]
    case = next(c for c in cases if c["workload"] == workload and c["metric"] == metric)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X).tobytes())
    h.update(np.ascontiguousarray(L).tobytes())
    assert h.hexdigest() == case["data_sha256"], "the seeded generator no longer gives the golden's data"
    return case
