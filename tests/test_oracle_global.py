"""Pins of the oracle's subsampled global estimators (Section 4.2): the row
draw, gl-s (Eq. 8) and gl-pps-s / gl-uni-s (Eq. 10).  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2607_01993_amd import synth


def brute_silhouette(X, L, k):
    """Eqs. 1-2 by a plain double loop (independent of the oracle)."""
    n = X.shape[0]
    s = np.zeros(n)
    sizes = np.bincount(L, minlength=k)
    for i in range(n):
        if sizes[L[i]] == 1:
            continue
        sums = np.zeros(k)
        for j in range(n):
            sums[L[j]] += math.sqrt(sum((float(X[i, c]) - float(X[j, c])) ** 2 for c in range(X.shape[1])))
        a = sums[L[i]] / (sizes[L[i]] - 1)
        b = min(sums[j] / sizes[j] for j in range(k) if j != L[i] and sizes[j] > 0)
        s[i] = (b - a) / max(a, b) if max(a, b) > 0 else 0.0
    return s


def test_draw_rows_is_floor_of_u_times_n():
    """The integer map equals floor(U * n) of the published 53-bit uniform
    (pinned by the Philox known-answer tests) wherever the float product is
    not within one ulp of an integer."""
    for n in (1, 2, 7, 1000, 999_983, (1 << 30)):
        m = 4000
        r = oracle.draw_rows(11, n, m)
        u = oracle.uniform53(11, np.arange(m), oracle.STREAM_ROWS)
        f = u * n
        safe = np.abs(f - np.round(f)) > n * 2.0 ** -50   # a few ulps of the product
        assert safe.mean() > 0.99
        assert np.all(r[safe] == np.floor(f[safe]).astype(np.int64))
        assert r.min() >= 0 and r.max() < n


def test_draw_rows_uniform_and_independent():
    n, m = 50, 200_000
    r = oracle.draw_rows(3, n, m)
    cnt = np.bincount(r, minlength=n)
    chi2 = float(((cnt - m / n) ** 2 / (m / n)).sum())
    assert chi2 < 49 + 6 * math.sqrt(2 * 49)            # 49 dof, ~6 sigma
    # with replacement: the number of distinct values among 40 draws from 50
    ds = [np.unique(oracle.draw_rows(s, 50, 40)).shape[0] for s in range(400)]
    expect = 50 * (1 - (1 - 1 / 50) ** 40)            # about 27.7
    assert abs(np.mean(ds) - expect) < 0.5
    # draws of different seeds and of consecutive counters are uncorrelated
    a = oracle.draw_rows(1, 1000, 5000).astype(float)
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 0.06
    b = oracle.draw_rows(2, 1000, 5000).astype(float)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.06


def test_gl_s_is_the_mean_of_exact_values_over_the_draws():
    """Eq. 8 against a brute-force silhouette; m > n forces duplicates, each
    counted in the mean."""
    X, L = synth.tiny_case(60, 3, 3, seed=4)
    s = brute_silhouette(X, L, 3)
    m = 150
    res = oracle.gl_s(X, L, 3, "eucl", m, seed=5)
    rows = oracle.draw_rows(5, 60, m)
    assert np.array_equal(res["rows"], rows)
    assert np.unique(rows).shape[0] < m
    np.testing.assert_allclose(res["s"], s[rows], atol=1e-12)
    assert abs(res["mean"] - s[rows].sum() / m) < 1e-12


def test_gl_pps_s_reduces_to_gl_s_when_clusters_are_taken_whole():
    """t >= max |C_j|: every p is 1, s_hat = s, so Eq. 10 equals Eq. 8 on the
    same draws."""
    X, L = synth.tiny_case(300, 4, 3, seed=6)
    g1 = oracle.gl_s(X, L, 3, "eucl", 80, seed=9)
    g2 = oracle.gl_pps_s(X, L, 3, "eucl", t=1000, delta=0.01, seed=1, m=80, rows_seed=9)
    np.testing.assert_allclose(g2["s"], g1["s"], atol=1e-12)
    assert abs(g2["mean"] - g1["mean"]) < 1e-12


@pytest.mark.parametrize("sampler", ["pps", "uni"])
def test_gl_pps_s_is_unbiased_for_s_hat_2(sampler):
    """The lemma after Eq. 10: over the row draws (Phase 1 fixed), the mean of
    s_bar is s_hat_2; z-test over 300 row seeds."""
    X, L = synth.tiny_case(2000, 5, 4, seed=8)
    smp = oracle.sample(X, L, 4, "eucl", 32, 0.01, 3, sampler)
    full = oracle.estimate(X, L, 4, "eucl", smp)
    s_all = full["s"]
    m = 25
    means = []
    for rs in range(300):
        rows = oracle.draw_rows(1000 + rs, 2000, m)
        means.append(s_all[rows].sum() / m)
    means = np.array(means)
    se = s_all.std() / math.sqrt(m) / math.sqrt(len(means))
    assert abs(means.mean() - full["mean"]) < 5 * se
    # one draw through the estimator itself gives the same s_bar
    g = oracle.gl_pps_s(X, L, 4, "eucl", t=32, delta=0.01, seed=3, m=m, rows_seed=1000, sampler=sampler)
    assert abs(g["mean"] - means[0]) < 1e-12


def test_hoeffding_size_bounds_the_subsampling_error():
    """With m = m_for(eps2, delta2) the draws miss s_hat_2 by more than eps2 in
    at most a delta2 fraction of row seeds (plus slack)."""
    X, L = synth.tiny_case(3000, 4, 5, seed=12)
    smp = oracle.sample(X, L, 5, "eucl", 40, 0.01, 2, "pps")
    full = oracle.estimate(X, L, 5, "eucl", smp)
    eps2, delta2 = 0.1, 0.1
    m = oracle.m_for(eps2, delta2)
    assert m == math.ceil(200 * math.log(20))
    miss = 0
    for rs in range(200):
        rows = oracle.draw_rows(rs, 3000, m)
        miss += abs(full["s"][rows].mean() - full["mean"]) > eps2
    assert miss <= 0.1 * 200


def brute_coh_sep(X, L, k):
    """Appendix B's definitions over explicit pairs (independent of W)."""
    n = X.shape[0]
    intra = inter = 0.0
    n_intra = n_inter = 0
    for i in range(n):
        for j in range(i + 1, n):
            dv = math.sqrt(sum((float(X[i, c]) - float(X[j, c])) ** 2 for c in range(X.shape[1])))
            if L[i] == L[j]:
                intra += dv
                n_intra += 1
            else:
                inter += dv
                n_inter += 1
    return intra / n_intra, inter / n_inter


def test_coh_sep_from_exact_weights_matches_pair_definitions():
    X, L = synth.tiny_case(90, 3, 4, seed=14)
    ex = oracle.exact(X, L, 4, "eucl")
    cs = oracle.coh_sep_from_weights(ex["W"], L, ex["sizes"])
    coh, sep = brute_coh_sep(X, L, 4)
    assert abs(cs["coh"] - coh) < 1e-12 * coh
    assert abs(cs["sep"] - sep) < 1e-12 * sep
    sizes = np.bincount(L, minlength=4)
    assert cs["coh_den"] == sum(c * (c - 1) // 2 for c in sizes)
    assert cs["sep_den"] == (90 * 90 - (sizes ** 2).sum()) // 2


def test_coh_sep_estimates_are_unbiased_in_the_numerators():
    """E[W_hat] = W (Horvitz-Thompson), so the numerators of the estimates are
    unbiased; z-test over 300 seeds."""
    X, L = synth.tiny_case(600, 4, 3, seed=15)
    ex = oracle.exact(X, L, 3, "eucl")
    truth = oracle.coh_sep_from_weights(ex["W"], L, ex["sizes"])
    vals = []
    for seed in range(300):
        smp = oracle.sample(X, L, 3, "eucl", 24, 0.01, seed, "pps")
        est = oracle.estimate(X, L, 3, "eucl", smp)
        cs = oracle.coh_sep_from_weights(est["W"], L, smp["sizes"])
        vals.append((cs["coh"], cs["sep"]))
    vals = np.array(vals)
    for c, key in ((0, "coh"), (1, "sep")):
        se = vals[:, c].std() / math.sqrt(len(vals))
        assert abs(vals[:, c].mean() - truth[key]) < 5 * se + 1e-12


def test_sweep_best_matches_the_exact_best():
    """Voronoi clusterings of blob data: the PPS estimates pick the same
    clustering as the exact global silhouette (values far apart here:
    0.61, 0.73, 0.24, 0.26, 0.14), and the subsampled means stay close."""
    X, L0 = synth.tiny_case(1200, 4, 4, seed=16, sigma=(0.2, 0.4))
    ks = [2, 3, 4, 5, 6]
    sets = [synth.voronoi_labels(X, synth.voronoi_centers(1200, k, (16, k))) for k in ks]
    exact = [oracle.exact(X, L, k, "eucl")["mean"] for L, k in zip(sets, ks)]
    res = oracle.sweep(X, sets, ks, "eucl", t=64, delta=0.01, seed=1)
    assert int(np.argmax(exact)) == res["best"]
    assert np.max(np.abs(res["means"] - np.array(exact))) < 0.05
    sub = oracle.sweep(X, sets, ks, "eucl", t=64, delta=0.01, seed=1, m=600)
    assert np.max(np.abs(sub["means"] - res["means"])) < 0.1
