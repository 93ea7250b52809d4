"""Phase 1 when the initial sample outgrows the capacity that the device-built
W(e_bar) work items get (64k + 1024 rows of F0): with delta = 1e-300 the rate
(2/|C_j|) ln(5k/delta) has ln(5k/delta) = 693, so every cluster larger than t
draws about 1,400 initial rows.  The eager request then runs Phase 1 again
with exact, host-built items and must still match the oracle (sample sets,
F0, W, scores); the captured graph flags such a clustering and re-runs it on
the eager path."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_01993_amd import native, synth
from parity_util import S_ATOL, assert_same_sets, compare_scores, dev

pytestmark = pytest.mark.gpu

DELTA = 1e-300


def test_eager_request_with_an_oversized_initial_sample():
    n, k, t, seed = 20000, 4, 64, 3
    X, L = synth.tiny_case(n, 8, k, seed=41)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, k, "eucl", "fp32", t=t, delta=DELTA, seed=seed)
    S, per = native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, k, "eucl", t, DELTA, seed, "pps")
    assert sum(f.shape[0] for f in smp["F0"]) > 64 * k + 1024  # past the capacity
    assert S == view["S"] and per.tolist() == [f.shape[0] for f in smp["F"]]
    assert_same_sets(smp, view, n, seed, "pps", t)
    for j in range(k):
        f0 = view["f0_gid"][view["f0_offsets"][j]:view["f0_offsets"][j + 1]]
        assert np.array_equal(f0, smp["F0"][j])
        np.testing.assert_allclose(view["f0_W"][view["f0_offsets"][j]:view["f0_offsets"][j + 1]],
                                   smp["W0"][j], rtol=1e-13)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-13)
    est = oracle.estimate(X, L, k, "eucl", smp)
    gpu = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    compare_scores(gpu, est)
    assert abs(gpu["mean"] - est["mean"]) <= S_ATOL


def test_graph_reruns_a_clustering_with_an_oversized_initial_sample():
    n, ks = 12000, [3, 5]
    X = synth.exp_blobs(n, 16, 6, seed=42)
    sets = [synth.voronoi_labels(X, synth.voronoi_centers(n, k, (42, k))) for k in ks]
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(np.stack(sets)).cuda().contiguous()
    g = native.SweepGraph(Xd, Ld, ks, "eucl", "bf16", t=48, delta=DELTA, seed=9, chains=2)
    got = g.run()
    g.close()
    ref = []
    for i, k in enumerate(ks):
        ctx = native.silh_sample_init(Xd, Ld[i], k, "eucl", "bf16", t=48, delta=DELTA, seed=9)
        native.silh_pps_sample(ctx)
        ref.append(native.silh_scores(ctx, a=False, b=False, s=False)["mean"])
        native.silh_destroy(ctx)
    assert got["reruns"] == len(ks)
    assert got["status"] == ["SILH_OK"] * len(ks)
    assert np.array_equal(got["means"], np.array(ref))
