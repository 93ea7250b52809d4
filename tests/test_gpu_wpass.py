"""Phase 1's W pass for rows of 65..128 coordinates, which streams each
member row from memory against groups of initial-sample rows in LDS
(Algorithm 1, Phase 1: W(e_bar) as the sum of e_bar's distances to its
cluster).  Against the float64 oracle: the initial sample ids exactly, W and
the inclusion probabilities to 1e-13, and the sample sets bit for bit, for
every metric, with a row length that takes the vector loads (128) and one
that does not (99)."""
import numpy as np
import pytest

import oracle
from paper_2607_01993_amd import native, synth
from parity_util import assert_same_sets, dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("metric", ["eucl", "cos", "manh", "canb"])
@pytest.mark.parametrize("d", [99, 128])
def test_streamed_w_pass(metric, d):
    n, k, t, seed = 3000, 4, 64, 3
    X, L = synth.tiny_case(n, d, k, seed=d)
    print(f"w pass metric={metric} d={d} n={n} k={k} t={t}", flush=True)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, k, metric, "fp32", t=t, delta=0.01, seed=seed)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, k, metric, t, 0.01, seed)
    assert_same_sets(smp, view, n, seed, "pps", t)
    for j in range(k):
        lo, hi = view["f0_offsets"][j], view["f0_offsets"][j + 1]
        assert hi > lo  # every cluster exceeds t, so its W pass runs
        assert np.array_equal(view["f0_gid"][lo:hi], smp["F0"][j])
        np.testing.assert_allclose(view["f0_W"][lo:hi], smp["W0"][j], rtol=1e-13)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-13)
    native.silh_destroy(ctx)
