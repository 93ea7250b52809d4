"""The k-sweep at its full size: n = 5e5 rows of d = 64 exponential blobs,
Voronoi clusterings for k = 2..257 (labels computed on the device), t = 128.
The captured graph and the worker-stream sweep give the same 256 means bit
for bit; for three clusterings the sample sets equal the oracle's and the
scores of sampled rows match it (float32 Euclidean and Canberra)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_01993_amd import native, sweep
from parity_util import assert_same_sets, compare_scores

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sweep_case():
    X, L, ks = sweep.build()   # seeded; labels on the device
    return X, L, ks


def test_full_sweep_graph_equals_worker_streams(sweep_case):
    X, L, ks = sweep_case
    print(f"full sweep: n={X.shape[0]} d={X.shape[1]} K={len(ks)} eucl bf16", flush=True)
    ref = native.silh_sweep(X, L, ks, "eucl", "bf16", t=128, seed=3, workers=4)
    g = native.SweepGraph(X, L, ks, "eucl", "bf16", t=128, seed=3, chains=4)
    got = g.run()
    g.close()
    assert got["status"] == ["SILH_OK"] * len(ks)
    assert np.array_equal(got["means"], ref["means"])
    assert got["best"] == ref["best"]


@pytest.mark.parametrize("metric", ["eucl", "canb"])
def test_full_sweep_clusterings_against_the_oracle(sweep_case, metric):
    X, L, ks = sweep_case
    Xh = X.cpu().numpy()
    n = Xh.shape[0]
    rows = np.sort(np.concatenate([np.random.default_rng(5).choice(n, 300, replace=False), [0, n - 1]]))
    for k in (2, 34, 257):
        i = ks.index(k)
        print(f"clustering k={k} metric={metric}", flush=True)
        Lh = L[i].cpu().numpy()
        ctx = native.silh_sample_init(X, L[i], k, metric, "fp32", t=128, delta=0.01, seed=3)
        native.silh_pps_sample(ctx)
        view = native.silh_sample_view(ctx)
        smp = oracle.sample(Xh, Lh, k, metric, 128, 0.01, 3, "pps")
        assert_same_sets(smp, view, n, 3, "pps", 128)
        gpu = native.silh_scores(ctx)
        native.silh_destroy(ctx)
        est = oracle.estimate(Xh, Lh, k, metric, smp, rows=rows)
        compare_scores(gpu, est, rows=rows, prec="fp32")
    del Xh
    torch.cuda.empty_cache()
