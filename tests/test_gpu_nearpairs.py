"""Euclidean pairs prone to cancellation, against the float64 oracle.

The matrix-core kernels evaluate |x - y|^2 as |x~|^2 + |y~|^2 - 2 x~.y~ with
both points centred on a centre of the cluster's sample.  When a cluster is
two tight blobs far apart (its centre lies between them, far from every one
of its points) the near pairs inside one blob carry a rounding error of the
size of |x~|^2 times the operand precision, far above their own squared
distance; near-duplicate rows inside wide blobs are the same case for single
pairs.  Those pairs must be evaluated again from the float32 rows: the
float32 bars (a_hat, b_hat to 1e-5 relative) and the bf16 bars (s_hat to
1e-2, the mean to 1e-3) hold only if they are.  Inputs: synth.split_blobs
(half the rows in cluster 0, a common offset of 1000 in every coordinate).
"""
import numpy as np
import pytest

import oracle
from parity_util import assert_same_sets, compare_scores, dev, mean_tol
from paper_2607_01993_amd import native, synth

pytestmark = pytest.mark.gpu

CASES = [("fp32", 32, 0.001, 0.0), ("bf16", 32, 0.001, 0.0), ("fp32", 64, 0.001, 0.0),
         ("bf16", 128, 0.001, 0.0), ("fp32", 128, 0.01, 0.0), ("bf16", 256, 0.001, 0.0),
         ("fp32", 16, 5.0, 1e-4), ("bf16", 64, 5.0, 1e-4)]


@pytest.mark.parametrize("prec,d,tight,dup", CASES)
def test_split_cluster_near_pairs(prec, d, tight, dup):
    n, k, t, seed = 4000, 3, 64, 11
    X, L = synth.split_blobs(n, d, k, seed=d, tight=tight, dup=dup)
    print(f"case prec={prec} d={d} tight={tight} dup={dup}", flush=True)
    smp = oracle.sample(X, L, k, "eucl", t, 0.01, seed)
    est = oracle.estimate(X, L, k, "eucl", smp)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, k, "eucl", prec, t=t, delta=0.01, seed=seed)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    assert_same_sets(smp, view, n, seed, "pps", t)
    gpu = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    compare_scores(gpu, est, prec=prec)
    assert abs(gpu["mean"] - est["mean"]) <= mean_tol(prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_split_cluster_exact(prec):
    """The exact silhouette (every pair of the dataset) on the same data."""
    n, d, k = 3000, 32, 3
    X, L = synth.split_blobs(n, d, k, seed=5, tight=0.001)
    ex = oracle.exact(X, L, k, "eucl")
    Xd, Ld = dev(X, L)
    gpu = native.silh_exact(Xd, Ld, k, "eucl", prec)
    compare_scores(gpu, ex, prec=prec)
    assert abs(gpu["mean"] - ex["mean"]) <= mean_tol(prec)
