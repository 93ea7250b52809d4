"""GPU parity: the HIP path (through the C ABI) against the float64 CPU oracle.

Bars: sample index sets bit-exact (a decision may differ only where the
uniform lies within 1e-12 of the oracle's rate: both sides decide in float64
but sum W(e_bar) in different orders); float32 a_hat, b_hat within 1e-5
relative; s_hat and the mean within 4e-5 absolute (Lemma 2 with rho = 1e-5:
4 rho / (1 - rho))."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2607_01993_amd import native, synth
from parity_util import (A_B_RTOL, FP8_S_ATOL, LOWP_MEAN_ATOL, LOWP_S_ATOL, S_ATOL,  # noqa: F401
                         assert_same_sets, compare_scores, dev, golden_mean, mean_tol)

pytestmark = pytest.mark.gpu


# (metric, prec) pairs with a Phase-2 kernel: float32 on the matrix cores for
# Euclidean / cosine, float32 on the vector ALUs for all, bf16 for Euclidean / cosine
COMBOS = [("eucl", "fp32"), ("eucl", "fp32_valu"), ("eucl", "bf16"), ("cos", "fp32"),
          ("cos", "fp32_valu"), ("cos", "bf16"), ("manh", "fp32"), ("canb", "fp32")]


# ---------------------------------------------------------------------------
def test_philox_bit_exact():
    for seed in (0, 1, 0x1234_5678_9ABC_DEF0):
        for stream in (0, 1, 2):
            g0 = 0 if seed else (1 << 32) - 5   # crosses the 32-bit boundary of the id
            u = native.silh_philox_uniform(seed, g0, 1 << 18, stream).cpu().numpy()
            ref = oracle.uniform53(seed, np.arange(g0, g0 + (1 << 18), dtype=np.uint64), stream)
            assert np.array_equal(u, ref)


@pytest.mark.parametrize("sampler", ["pps", "uni"])
def test_small_config_parity(sampler):
    """n=2,000, d=8, k=4 Gaussian blobs, Euclidean, t=64, seed 0."""
    X, L = synth.config_small()
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 4, "eucl", t=64, delta=0.01, seed=0, sampler=sampler)
    S, per = native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, 4, "eucl", 64, 0.01, 0, sampler)
    assert S == view["S"] and per.tolist() == [f.shape[0] for f in smp["F"]]
    assert_same_sets(smp, view, X.shape[0], 0, sampler, 64)
    if sampler == "pps":
        for j in range(4):
            f0 = view["f0_gid"][view["f0_offsets"][j]:view["f0_offsets"][j + 1]]
            assert np.array_equal(f0, smp["F0"][j])
            np.testing.assert_allclose(view["f0_W"][view["f0_offsets"][j]:view["f0_offsets"][j + 1]],
                                       smp["W0"][j], rtol=1e-13)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-13)
    est = oracle.estimate(X, L, 4, "eucl", smp)
    gpu = native.silh_scores(ctx)
    compare_scores(gpu, est)
    assert abs(gpu["mean"] - est["mean"]) <= S_ATOL
    W = native.silh_weighted_sums(ctx).cpu().numpy()
    np.testing.assert_allclose(W, est["W"], rtol=A_B_RTOL)
    native.silh_destroy(ctx)


def test_small_config_exact():
    X, L = synth.config_small()
    Xd, Ld = dev(X, L)
    gpu = native.silh_exact(Xd, Ld, 4, "eucl")
    ref = oracle.exact(X, L, 4, "eucl")
    compare_scores(gpu, ref)
    assert abs(gpu["mean"] - ref["mean"]) <= S_ATOL


def _ragged_case(metric, n=3001, d=13, k=6, seed=5):
    # uneven clusters, one singleton (id 4) and one empty cluster (id 5)
    X, L = synth.tiny_case(n, d, 4, seed=seed)
    L = L.copy()
    L[17] = 4
    if metric == "canb":
        X = np.abs(X).astype(np.float32)
        X[:5, :3] = 0.0                      # 0/0 coordinates
    if metric == "cos":
        X[3] = 0.0                           # a zero row
    return X, L, k


@pytest.mark.parametrize("metric,prec", COMBOS)
@pytest.mark.parametrize("sampler", ["pps", "uni"])
def test_all_metrics_ragged(metric, prec, sampler):
    X, L, k = _ragged_case(metric)
    Xd, Ld = dev(X, L)
    t = 40
    ctx = native.silh_sample_init(Xd, Ld, k, metric, prec, t=t, delta=0.01, seed=77, sampler=sampler)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, k, metric, t, 0.01, 77, sampler)
    assert_same_sets(smp, view, X.shape[0], 77, sampler, t)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-12)
    est = oracle.estimate(X, L, k, metric, smp)
    gpu = native.silh_scores(ctx)
    compare_scores(gpu, est, prec=prec)
    assert abs(gpu["mean"] - est["mean"]) <= mean_tol(prec)
    s = gpu["s"].cpu().numpy()
    assert s[17] == 0.0                               # singleton
    W = native.silh_weighted_sums(ctx).cpu().numpy()
    assert np.all(W[:, 5] == 0.0)                     # empty cluster
    # elementwise weights: relative bar, plus an absolute floor for the cosine
    # self-distance, which is rounding-level (about 1e-16) in the oracle
    if prec != "bf16":
        np.testing.assert_allclose(W[:, :5], est["W"][:, :5], rtol=A_B_RTOL, atol=1e-9)
    else:
        np.testing.assert_allclose(W[:, :5], est["W"][:, :5], rtol=1e-2, atol=1e-6)
    native.silh_destroy(ctx)


@pytest.mark.parametrize("metric,prec", COMBOS)
def test_exact_all_metrics(metric, prec):
    X, L, k = _ragged_case(metric, n=1500, d=7)
    Xd, Ld = dev(X, L)
    gpu = native.silh_exact(Xd, Ld, k, metric, prec)
    ref = oracle.exact(X, L, k, metric)
    compare_scores(gpu, ref, prec=prec)
    assert abs(gpu["mean"] - ref["mean"]) <= mean_tol(prec)


@pytest.mark.parametrize("metric,prec", [("eucl", "fp32"), ("cos", "fp32"), ("eucl", "bf16"),
                                         ("cos", "bf16")])
@pytest.mark.parametrize("d", [3, 16, 50, 128])
def test_mfma_dims(metric, prec, d):
    """Every padded dimension of the MFMA kernel, with n not a multiple of the
    128-row block."""
    X, L = synth.tiny_case(1000 + 37 * d, d, 5, seed=d)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 5, metric, prec, t=33, seed=d)
    native.silh_pps_sample(ctx)
    smp = oracle.sample(X, L, 5, metric, 33, 0.01, d)
    est = oracle.estimate(X, L, 5, metric, smp)
    gpu = native.silh_scores(ctx)
    compare_scores(gpu, est, prec=prec)
    assert abs(gpu["mean"] - est["mean"]) <= mean_tol(prec)
    native.silh_destroy(ctx)


@pytest.mark.parametrize("metric,prec", COMBOS)
@pytest.mark.parametrize("d", [200, 256])
def test_wide_rows(metric, prec, d):
    """d > 128: Phase 1 and the vector-ALU Phase 2 keep rows in LDS, bf16
    stays on the matrix cores; sample sets bit-exact, scores to the bars,
    with a singleton cluster and n not a multiple of any block."""
    X, L = synth.tiny_case(2300 + d, d, 5, seed=d + 1)
    L = L.copy()
    L[L == 4] = 3
    L[9] = 4
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 5, metric, prec, t=40, seed=d)
    native.silh_pps_sample(ctx)
    smp = oracle.sample(X, L, 5, metric, 40, 0.01, d)
    view = native.silh_sample_view(ctx)
    assert_same_sets(smp, view, X.shape[0], d, "pps", 40)
    np.testing.assert_allclose(view["f0_W"], np.concatenate([smp["W0"][j] for j in range(5)]),
                               rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-12)
    est = oracle.estimate(X, L, 5, metric, smp)
    gpu = native.silh_scores(ctx)
    compare_scores(gpu, est, prec=prec)
    assert abs(gpu["mean"] - est["mean"]) <= mean_tol(prec)
    native.silh_destroy(ctx)


def test_wide_rows_fp8_and_exact():
    X, L = synth.vmf_blobs(3000, 256, 4, seed=7, kappa=60.0)
    Xd, Ld = dev(X, L)
    gpu = native.silh_exact(Xd, Ld, 4, "cos", "fp8")
    ref = oracle.exact(X, L, 4, "cos")
    assert abs(gpu["mean"] - ref["mean"]) <= LOWP_MEAN_ATOL
    compare_scores(gpu, ref, prec="fp8")
    gpu = native.silh_exact(Xd, Ld, 4, "eucl", "bf16")
    ref = oracle.exact(X, L, 4, "eucl")
    compare_scores(gpu, ref, prec="bf16")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("d", [16, 64, 128])
def test_cosine_directional(prec, d):
    """Unit-norm vMF blobs (the directional workload) at every MFMA operand
    type, against the float64 oracle on all rows."""
    X, L = synth.vmf_blobs(12_000, d, 8, seed=d, kappa=50.0)
    Xd, Ld = dev(X, L)
    if prec == "fp8" and d < 64:
        with pytest.raises(native.SilhError) as e:
            native.silh_sample_init(Xd, Ld, 8, "cos", prec, t=256, seed=3)
        assert e.value.name == "SILH_E_UNSUPPORTED"
        return
    ctx = native.silh_sample_init(Xd, Ld, 8, "cos", prec, t=256, seed=3)
    native.silh_pps_sample(ctx)
    smp = oracle.sample(X, L, 8, "cos", 256, 0.01, 3)
    view = native.silh_sample_view(ctx)
    assert_same_sets(smp, view, X.shape[0], 3, "pps", 256)
    est = oracle.estimate(X, L, 8, "cos", smp)
    gpu = native.silh_scores(ctx)
    assert abs(gpu["mean"] - est["mean"]) <= mean_tol(prec)
    compare_scores(gpu, est, prec=prec)
    native.silh_destroy(ctx)


def test_fp8_exact_directional():
    """Exact cosine silhouette with fp8 operands on vMF blobs."""
    X, L = synth.vmf_blobs(3000, 128, 4, seed=5, kappa=50.0)
    Xd, Ld = dev(X, L)
    gpu = native.silh_exact(Xd, Ld, 4, "cos", "fp8")
    ref = oracle.exact(X, L, 4, "cos")
    assert abs(gpu["mean"] - ref["mean"]) <= LOWP_MEAN_ATOL
    compare_scores(gpu, ref, prec="fp8")


def test_fp8_rejected_for_other_metrics():
    X, L = synth.tiny_case(300, 4, 3, seed=1)
    Xd, Ld = dev(X, L)
    for metric in ("eucl", "manh", "canb", "cos"):  # cos: d = 4 < 64
        with pytest.raises(native.SilhError) as e:
            native.silh_sample_init(Xd, Ld, 3, metric, "fp8", t=10)
        assert e.value.name == "SILH_E_UNSUPPORTED"


def test_large_t_equals_exact():
    """Algorithm 1: t >= max |C_j| takes every cluster whole (p = 1)."""
    X, L = synth.tiny_case(1200, 5, 3, seed=9)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 3, "eucl", t=5000, seed=1)
    S, _ = native.silh_pps_sample(ctx)
    assert S == 1200
    view = native.silh_sample_view(ctx)
    assert np.all(view["p"] == 1.0) and view["F0"] == 0
    est = native.silh_scores(ctx)
    ex = native.silh_exact(Xd, Ld, 3, "eucl")
    for key in ("a", "b", "s"):
        assert torch.equal(est[key], ex[key])
    assert est["mean"] == ex["mean"]
    native.silh_destroy(ctx)


def test_resample_is_deterministic():
    X, L = synth.tiny_case(5000, 6, 5, seed=3)
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 5, "manh", t=30, seed=11)
    native.silh_pps_sample(ctx)
    v1 = native.silh_sample_view(ctx)
    r1 = native.silh_scores(ctx)
    native.silh_pps_sample(ctx)
    v2 = native.silh_sample_view(ctx)
    r2 = native.silh_scores(ctx)
    assert np.array_equal(v1["gid"], v2["gid"]) and np.array_equal(v1["p"], v2["p"])
    assert torch.equal(r1["s"], r2["s"]) and r1["mean"] == r2["mean"]
    native.silh_destroy(ctx)


# ---------------------------------------------------------------------------
# error paths reachable from the host
# ---------------------------------------------------------------------------
def test_error_paths():
    X, L = synth.tiny_case(300, 3, 3, seed=1)
    Xd, Ld = dev(X, L)
    bad = Ld.clone()
    bad[10] = 3
    with pytest.raises(native.SilhError) as e:
        native.silh_sample_init(Xd, bad, 3, "eucl", t=10)
    assert e.value.name == "SILH_E_LABEL"
    neg = Ld.clone()
    neg[0] = -1
    with pytest.raises(native.SilhError) as e:
        native.silh_exact(Xd, neg, 3, "eucl")
    assert e.value.name == "SILH_E_LABEL"
    one = torch.zeros_like(Ld)
    with pytest.raises(native.SilhError) as e:
        native.silh_sample_init(Xd, one, 3, "eucl", t=10)
    assert e.value.name == "SILH_E_K"
    ctx = native.silh_sample_init(Xd, Ld, 3, "eucl", t=10)
    with pytest.raises(native.SilhError) as e:
        native.silh_scores(ctx)
    assert e.value.name == "SILH_E_STATE"
    with pytest.raises(native.SilhError) as e:
        native.silh_weighted_sums(ctx)
    assert e.value.name == "SILH_E_STATE"
    native.silh_pps_sample(ctx)
    native.silh_scores(ctx)
    native.silh_destroy(ctx)


def test_allocator_failure_reports_nomem():
    import ctypes
    lib = native.load_library()
    X, L = synth.tiny_case(300, 3, 3, seed=1)
    Xd, Ld = dev(X, L)
    p = native._params(300, 3, 3, "eucl", "fp32", "pps", 10, 0.0, 0.01, 0, use_torch_alloc=False)
    p.alloc = native.ALLOC_FN(lambda nbytes, user: None)
    p.free = native.FREE_FN(lambda ptr, user: None)
    out = ctypes.c_void_p()
    st = lib.silh_sample_init(ctypes.byref(p), ctypes.c_void_p(Xd.data_ptr()),
                              ctypes.c_void_p(Ld.data_ptr()), None, ctypes.byref(out))
    assert native.STATUS[st] == "SILH_E_NOMEM"
    assert not out.value
    torch.cuda.synchronize()


@pytest.mark.parametrize("fail_at", [1, 2, 3, 4])
def test_allocator_failure_mid_request(fail_at):
    """The allocator fails at its fail_at-th call (the index, the per-sampling
    buffers, the F0 buffers, the sample buffers): the failing call reports
    SILH_E_NOMEM, every block handed out is freed exactly once."""
    import ctypes
    lib = native.load_library()
    X, L = synth.tiny_case(3000, 5, 4, seed=2)
    Xd, Ld = dev(X, L)
    live, calls, freed_twice = {}, [0], []

    def alloc(nbytes, user):
        calls[0] += 1
        if calls[0] >= fail_at + 1:
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, user):
        if ptr not in live:
            freed_twice.append(ptr)
        live.pop(ptr, None)

    afn, ffn = native.ALLOC_FN(alloc), native.FREE_FN(free)
    p = native._params(3000, 5, 4, "eucl", "bf16", "pps", 64, 0.0, 0.01, 0, use_torch_alloc=False)
    p.alloc, p.free = afn, ffn
    out = ctypes.c_void_p()
    st = lib.silh_sample_init(ctypes.byref(p), ctypes.c_void_p(Xd.data_ptr()),
                              ctypes.c_void_p(Ld.data_ptr()), None, ctypes.byref(out))
    assert native.STATUS[st] == "SILH_OK"   # the index is the first call
    S = ctypes.c_int64()
    st = lib.silh_pps_sample(out, ctypes.byref(S), None)
    if fail_at <= 3:
        assert native.STATUS[st] == "SILH_E_NOMEM"
    else:
        assert native.STATUS[st] == "SILH_OK"
    lib.silh_destroy(out)
    torch.cuda.synchronize()
    assert not freed_twice
    assert not live


# ---------------------------------------------------------------------------
# full size: n=1e6, d=32, k=16 Zipf Gaussian blobs, t=256 (the benchmark workload)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def zipf_case():
    X, L = synth.config_zipf_gauss()
    return X, L


@pytest.mark.parametrize("metric,prec", [("eucl", "fp32"), ("eucl", "bf16"), ("manh", "fp32")])
def test_full_size_zipf(zipf_case, metric, prec):
    X, L = zipf_case
    k, t, seed = 16, 256, 1
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, k, metric, prec, t=t, delta=0.01, seed=seed)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    smp = oracle.sample(X, L, k, metric, t, 0.01, seed, "pps")
    assert_same_sets(smp, view, X.shape[0], seed, "pps", t)
    np.testing.assert_allclose(view["p"], smp["p"], rtol=1e-12)
    gpu = native.silh_scores(ctx)
    rows = np.random.default_rng(0).choice(X.shape[0], 1500, replace=False)
    rows = np.sort(np.concatenate([rows, [0, X.shape[0] - 1]]))
    est = oracle.estimate(X, L, k, metric, smp, rows=rows)
    compare_scores(gpu, est, rows=rows, prec=prec)
    # the mean over all n elements against the oracle's full-size value
    # (Eq. 9; tests/golden/fullsize_means.json, written from oracle/ only)
    gold = golden_mean(X, L, "zipf-gauss-blobs", metric)
    assert view["S"] == gold["S"]
    print(f"{metric}/{prec}: mean={gpu['mean']:.10f} oracle={gold['mean']:.10f} "
          f"|d|={abs(gpu['mean'] - gold['mean']):.2e}")
    assert abs(gpu["mean"] - gold["mean"]) <= mean_tol(prec)
    # the device mean is the float64 mean of the float64 scores; the float32
    # copies differ from those by at most 2^-24 each
    s = gpu["s"].cpu().numpy().astype(np.float64)
    assert abs(gpu["mean"] - math.fsum(s.tolist()) / s.shape[0]) < 1e-7
    native.silh_destroy(ctx)


# ---------------------------------------------------------------------------
# full size, directional: n=4e6, d=128, k=64 vMF(kappa=50) blobs with Zipf
# sizes, cosine, t=512 -- float32, bf16 and fp8 operands
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def vmf_case():
    X, L = synth.config_vmf_cos()
    smp = oracle.sample(X, L, 64, "cos", 512, 0.01, 2)
    rows = np.sort(np.concatenate([np.random.default_rng(1).choice(X.shape[0], 400, replace=False),
                                   [0, X.shape[0] - 1]]))
    est = oracle.estimate(X, L, 64, "cos", smp, rows=rows)
    gold = golden_mean(X, L, "vmf-blobs", "cos")
    return X, L, smp, rows, est, gold


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_full_size_vmf_cosine(vmf_case, prec):
    X, L, smp, rows, est, vmf_gold = vmf_case
    Xd, Ld = dev(X, L)
    ctx = native.silh_sample_init(Xd, Ld, 64, "cos", prec, t=512, delta=0.01, seed=2)
    native.silh_pps_sample(ctx)
    view = native.silh_sample_view(ctx)
    assert_same_sets(smp, view, X.shape[0], 2, "pps", 512)
    gpu = native.silh_scores(ctx)
    compare_scores(gpu, est, rows=rows, prec=prec)
    s = gpu["s"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(s) <= 1.0)
    assert abs(gpu["mean"] - math.fsum(s.tolist()) / s.shape[0]) < 1e-7
    # the mean over all n = 4e6 elements against the oracle's full-size value
    # (Eq. 9; tests/golden/fullsize_means.json, written from oracle/ only)
    gold = vmf_gold
    assert view["S"] == gold["S"]
    print(f"{prec}: mean={gpu['mean']:.10f} oracle={gold['mean']:.10f} |d|={abs(gpu['mean'] - gold['mean']):.2e}")
    assert abs(gpu["mean"] - gold["mean"]) <= mean_tol(prec)
    native.silh_destroy(ctx)
    del Xd, Ld
    torch.cuda.empty_cache()
