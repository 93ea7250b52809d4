"""GPU parity of the cohesion / separation estimates (Appendix B) against the
float64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2607_01993_amd import native, synth
from parity_util import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("metric,prec", [("eucl", "fp32"), ("eucl", "bf16"), ("cos", "fp32"), ("manh", "fp32"),
                                         ("canb", "fp32")])
def test_coh_sep_parity(metric, prec):
    X, L = synth.tiny_case(3000, 6, 5, seed=51)
    k, t, seed = 6, 64, 3            # cluster id 5 stays empty
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, k, metric, prec, "pps", t=t, seed=seed)
    native.silh_pps_sample(ctx)
    W = native.silh_weighted_sums(ctx)
    given = native.silh_coh_sep(ctx, W)
    own = native.silh_coh_sep(ctx)          # the library computes W_hat itself
    native.silh_destroy(ctx)
    smp = oracle.sample(X, L, k, metric, t, 0.01, seed, "pps")
    est = oracle.estimate(X, L, k, metric, smp)
    ref = oracle.coh_sep_from_weights(est["W"], L, smp["sizes"])
    tol = 1e-5 if prec == "fp32" else 2e-3
    for key in ("coh", "sep"):
        assert abs(given[key] - ref[key]) <= tol * ref[key], (key, given[key], ref[key])
        assert given[key] == own[key]


def test_coh_sep_exact_when_clusters_are_whole():
    X, L = synth.tiny_case(1200, 4, 3, seed=52)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 3, "eucl", "fp32", "pps", t=5000, seed=1)
    native.silh_pps_sample(ctx)
    got = native.silh_coh_sep(ctx)
    native.silh_destroy(ctx)
    ex = oracle.exact(X, L, 3, "eucl")
    ref = oracle.coh_sep_from_weights(ex["W"], L, ex["sizes"])
    assert abs(got["coh"] - ref["coh"]) <= 1e-5 * ref["coh"]
    assert abs(got["sep"] - ref["sep"]) <= 1e-5 * ref["sep"]


def test_coh_sep_requires_a_sample():
    X, L = synth.tiny_case(300, 3, 3, seed=2)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 3, "eucl", "fp32", t=16, seed=1)
    with pytest.raises(native.SilhError) as e:
        native.silh_coh_sep(ctx)
    assert e.value.name == "SILH_E_STATE"
    native.silh_destroy(ctx)
