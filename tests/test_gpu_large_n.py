"""A clustering with more rows than one pass of the int32 scan sums inside
its apply kernel (2,048 tiles of 2,048 rows): n = 4.5e6 takes the path with
the separate scan of the tile sums, in the request's compactions and in the
row-subset path.  Sample sets equal the oracle's (so do the inclusion
probabilities), scores of sampled rows match it, and the scores of a row
subset equal the full request's at those rows bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_01993_amd import native, synth
from parity_util import assert_same_sets, compare_scores

pytestmark = pytest.mark.gpu

N, D, K, T, SEED = 4_500_000, 4, 5, 32, 6


def test_large_n_sample_and_rows():
    assert N > 2048 * 2048
    X, L = synth.gaussian_blobs(N, D, K, seed=SEED, sizes=synth.zipf_sizes(N, K), sigma=(0.5, 2.0))
    print(f"large n: n={N} d={D} k={K} t={T}", flush=True)
    Xd, Ld = torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda()
    ctx = native.silh_sample_init(Xd, Ld, K, "eucl", "fp32", t=T, delta=0.01, seed=SEED)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, K, "eucl", T, 0.01, SEED, "pps")
    assert_same_sets(smp, view, N, SEED, "pps", T)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-12)
    full = native.silh_scores(ctx)
    rows = np.sort(np.concatenate([np.random.default_rng(3).choice(N, 600, replace=False), [0, N - 1]]))
    est = oracle.estimate(X, L, K, "eucl", smp, rows=rows)
    compare_scores(full, est, rows=rows)
    # the row-subset path marks and compacts all n rows with the same scan
    drawn = native.silh_draw_rows(11, N, 5000)
    sub = native.silh_scores_rows(ctx, drawn)
    r = drawn.cpu().numpy()
    for key in ("a", "b", "s"):
        assert np.array_equal(sub[key].cpu().numpy(), full[key].cpu().numpy()[r]), key
    native.silh_destroy(ctx)
    del Xd, Ld
    torch.cuda.empty_cache()
