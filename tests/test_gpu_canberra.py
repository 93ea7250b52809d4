"""Canberra on the vector ALUs: the coordinate-pair form (one reciprocal per
two coordinates) runs only where every coordinate of the wave's element rows
lies in [2^-62, 2^62] in magnitude and the sample row has none past 2^62;
elsewhere the per-coordinate guarded form runs.  Both against the float64
oracle at the float32 bars, on data that mixes the three cases."""
import numpy as np
import pytest

import oracle
from paper_2607_01993_amd import native
from parity_util import S_ATOL, assert_same_sets, compare_scores, dev

pytestmark = pytest.mark.gpu


def _mixed(n, d, k, seed):
    rng = np.random.default_rng(seed)
    X = (rng.exponential(1.0, size=(n, d)) + 0.1).astype(np.float32)
    X[:, : d // 2] *= np.where(rng.random((n, 1)) < 0.5, -1.0, 1.0).astype(np.float32)  # both signs
    L = (np.arange(n) * 7919 % k).astype(np.int32)
    # the first two 64-element waves hold coordinates past 2^62 (their
    # elements take the guarded form; sampled, these rows are flagged and
    # the other waves take the guarded form for them)
    X[:128, 3] = np.float32(3e19)
    # the third holds coordinates below 2^-62
    X[128:192, 5] = np.float32(1e-20)
    # the fourth exact zeros (0/0 against zero sample coordinates)
    X[192:256, 0] = 0.0
    X[192:256:2, 1] = 0.0
    return X, L


@pytest.mark.parametrize("d", [16, 32, 64])
def test_canberra_pair_form_and_guarded_rows(d):
    n, k, t, seed = 4000, 4, 512, 6
    X, L = _mixed(n, d, k, seed=d)
    print(f"canberra d={d} n={n} k={k} t={t}", flush=True)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, k, "canb", "fp32", t=t, delta=0.01, seed=seed)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, k, "canb", t, 0.01, seed)
    assert_same_sets(smp, view, n, seed, "pps", t)
    assert np.any(np.concatenate(smp["F"]) < 128)  # some flagged sample rows
    est = oracle.estimate(X, L, k, "canb", smp)
    gpu = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    compare_scores(gpu, est)
    assert abs(gpu["mean"] - est["mean"]) <= S_ATOL
