"""Degenerate inputs against the float64 oracle: two singleton clusters
(n = 2, d = 1), exact duplicates (zero distances), and a cluster of
identical points larger than t, where every W(e_bar) of the initial sample
is 0 and each is skipped (so gamma_e = 1/|C_j| and p = t/|C_j|)."""
import numpy as np
import pytest

import oracle
from parity_util import assert_same_sets, compare_scores, dev
from paper_2607_01993_amd import native

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("metric,prec", [("eucl", "fp32"), ("eucl", "bf16"), ("manh", "fp32")])
def test_two_singletons(metric, prec):
    X = np.array([[0.0], [1.0]], dtype=np.float32)
    L = np.array([0, 1], dtype=np.int32)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 2, metric, prec, t=4, seed=1)
    native.silh_pps_sample(ctx)
    res = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    # a singleton's silhouette is 0 (Section 2)
    assert res["s"].cpu().numpy().tolist() == [0.0, 0.0]
    assert res["mean"] == 0.0
    ex = oracle.exact(X, L, 2, metric)
    assert ex["s"].tolist() == [0.0, 0.0]


@pytest.mark.parametrize("metric,prec", [("eucl", "fp32"), ("eucl", "bf16"), ("manh", "fp32"),
                                         ("canb", "fp32")])
def test_duplicate_points(metric, prec):
    # clusters {1, 1, 1} and {6, 6}: within-cluster distances are exactly 0,
    # so a = 0 and s = 1 for every element
    X = np.array([[1.0], [1.0], [6.0], [1.0], [6.0]], dtype=np.float32)
    L = np.array([0, 0, 1, 0, 1], dtype=np.int32)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 2, metric, prec, t=8, seed=2)
    native.silh_pps_sample(ctx)
    res = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    ex = oracle.exact(X, L, 2, metric)
    np.testing.assert_array_equal(ex["s"], np.ones(5))
    np.testing.assert_array_equal(res["a"].cpu().numpy(), np.zeros(5, dtype=np.float32))
    np.testing.assert_array_equal(res["s"].cpu().numpy(), np.ones(5, dtype=np.float32))
    assert res["mean"] == 1.0


@pytest.mark.parametrize("metric,prec", [("eucl", "fp32"), ("eucl", "bf16"), ("cos", "fp32"), ("cos", "bf16"),
                                         ("cos", "fp32_valu"), ("manh", "fp32")])
def test_identical_cluster_larger_than_t(metric, prec):
    rng = np.random.default_rng(7)
    same = np.tile(np.array([[2.0, -1.0, 0.5]], dtype=np.float32), (200, 1))
    other = (rng.normal(size=(100, 3)) + 4.0).astype(np.float32)
    X = np.concatenate([same, other])
    L = np.concatenate([np.zeros(200, np.int32), np.ones(100, np.int32)])
    perm = rng.permutation(300)
    X, L = np.ascontiguousarray(X[perm]), np.ascontiguousarray(L[perm])
    t, seed = 10, 3
    smp = oracle.sample(X, L, 2, metric, t, 0.01, seed, "pps")
    assert len(smp["F0"][0]) > 0 and np.all(smp["W0"][0] == 0.0)
    np.testing.assert_allclose(smp["p"][L == 0], t / 200.0, rtol=0, atol=0)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 2, metric, prec, t=t, seed=seed)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    assert_same_sets(smp, view, 300, seed, "pps", t)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-13)
    gpu = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    est = oracle.estimate(X, L, 2, metric, smp)
    a = gpu["a"].cpu().numpy().astype(np.float64)
    compare_scores(gpu, est, prec=prec)
    # the identical points are 0 apart on the GPU too (a = 0 exactly); for
    # cosine both sides scale a row by the same float32 reciprocal norm
    assert np.all(a[L == 0] == 0.0)
