"""Block-shape autotuning of the matrix-core Phase-2 kernel: every shape
gives bit-identical a_hat, b_hat, s_hat and mean (the mean's partial sums are
per 128 elements, added in the same order, in every shape), and the tuner records a choice per key."""
import numpy as np
import pytest

from paper_2607_01993_amd import native, synth
from parity_util import dev

pytestmark = pytest.mark.gpu


def _run(X, L, k, metric, prec, mode):
    native.silh_set_tuning(mode)
    ctx = native.silh_sample_init(X, L, k, metric, prec, "pps", t=96, seed=4)
    S, _ = native.silh_pps_sample(ctx)
    res = native.silh_scores(ctx)
    view = native.silh_sample_view(ctx)
    native.silh_destroy(ctx)
    return res, S, view


@pytest.mark.parametrize("metric,prec,d", [("eucl", "fp32", 32), ("eucl", "bf16", 64), ("cos", "bf16", 16),
                                           ("cos", "fp32", 64), ("eucl", "bf16", 5), ("eucl", "bf16", 128),
                                           ("cos", "fp8", 128), ("eucl", "bf16", 32)])
def test_block_shapes_agree_bitwise(metric, prec, d):
    X, L = synth.tiny_case(7000, d, 5, seed=81)
    Xd, Ld = dev(X, L)
    try:
        outs = [_run(Xd, Ld, 5, metric, prec, mode) for mode in (2, 3, 4, 0, 1)]
        # mode 1 (last) measured this key; setting mode 1 again would forget it
        S_pad = sum(-(-c // 32) * 32 for c in np.diff(outs[0][2]["offsets"]))
        assert native.silh_tuning_choice(metric, prec, d, S_pad) in (1, 2, 3)
    finally:
        native.silh_set_tuning(1)
    ref = outs[0][0]
    for res, S, _ in outs[1:]:
        for x in ("a", "b", "s"):
            assert np.array_equal(res[x].cpu().numpy(), ref[x].cpu().numpy()), x
        assert res["mean"] == ref["mean"]


@pytest.mark.parametrize("metric,prec,d", [("eucl", "bf16", 64), ("cos", "bf16", 128)])
def test_graph_captures_the_tuned_shapes(metric, prec, d):
    """silh_graph_create tunes before it captures: the shape of every
    clustering is the autotuner's choice for the key of the request it was
    tuned on, and the replayed means equal the eager requests'."""
    n, K = 6000, 6
    X, L = synth.tiny_case(n, d, 4, seed=83)
    Xd, _ = dev(X, L)
    import torch
    ks = [2, 3, 5, 8, 13, 21]
    labels = torch.stack([torch.from_numpy(synth.voronoi_labels(X, synth.voronoi_centers(n, k, (9, k))))
                          for k in ks]).cuda().contiguous()
    native.silh_set_tuning(1)
    g = native.SweepGraph(Xd, labels, ks, metric, prec, t=48, seed=5, chains=2)
    try:
        for i in range(K):
            shape, S_pad = g.choice(i)
            assert S_pad > 0
            assert shape == native.silh_tuning_choice(metric, prec, d, S_pad), (i, shape, S_pad)
        out = g.run()
        for i, k in enumerate(ks):
            ctx = native.silh_sample_init(Xd, labels[i].contiguous(), k, metric, prec, "pps", t=48, delta=0.01, seed=5)
            native.silh_pps_sample(ctx)
            m = native.silh_scores(ctx, a=False, b=False, s=False)["mean"]
            native.silh_destroy(ctx)
            assert out["means"][i] == m
    finally:
        g.close()
