"""silh_exact_noalloc (the exact silhouette with the library's buffers in its
static device array) against silh_exact through the C ABI: two calls in a
row, the second on a smaller input, for the matrix-core and the vector-ALU
Phase-2 kernels, at the float32 bars of the parity tests (both sides run the
same kernels in the same precision)."""
import numpy as np
import pytest
import torch

from paper_2607_01993_amd import native, synth

pytestmark = pytest.mark.gpu

A_B_RTOL = 1e-5
S_ATOL = 4.0e-5


def _dev(X, L):
    return torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda()


def _same(ref, got):
    for key in ("a", "b"):
        np.testing.assert_allclose(got[key].cpu().numpy(), ref[key].cpu().numpy(), rtol=A_B_RTOL, atol=1e-30)
    s_ref, s_got = ref["s"].cpu().numpy(), got["s"].cpu().numpy()
    assert np.max(np.abs(s_got.astype(np.float64) - s_ref)) <= S_ATOL
    assert abs(got["mean"] - ref["mean"]) <= S_ATOL
    return bool(np.array_equal(s_got, s_ref)) and got["mean"] == ref["mean"]


@pytest.mark.parametrize("metric,prec,d", [("eucl", "bf16", 32), ("eucl", "fp32", 16), ("cos", "bf16", 64),
                                           ("manh", "fp32", 24), ("canb", "fp32", 200)])
def test_noalloc_matches_exact(metric, prec, d):
    sizes = [(40_000, 9), (12_345, 5)] if d <= 64 else [(6_000, 5), (2_500, 3)]
    for call, (n, k) in enumerate(sizes):
        X, L = synth.tiny_case(n, d, k, seed=31 + call)
        if metric == "canb":
            X = np.abs(X)
        Xd, Ld = _dev(X, L)
        print(f"case {metric} {prec} d={d} call={call} n={n} k={k}", flush=True)
        ref = native.silh_exact(Xd, Ld, k, metric, prec)
        got = native.silh_exact_noalloc(Xd, Ld, k, metric, prec)
        bitwise = _same(ref, got)
        print(f"  mean={got['mean']:.9f} exact={ref['mean']:.9f} bitwise={bitwise}", flush=True)


def test_noalloc_allocates_nothing():
    """After the first call (which loads the library's code object and its
    static array), further calls leave the device's free memory unchanged."""
    X, L = synth.tiny_case(30_000, 32, 8, seed=3)
    Xd, Ld = _dev(X, L)
    outs = {key: torch.empty(X.shape[0], dtype=torch.float32, device="cuda") for key in "abs"}
    lib = native.load_library()
    import ctypes
    p = native._params(X.shape[0], 32, 8, "eucl", "bf16", "pps", 1, 0.0, 0.5, 0, False)

    def call():
        m = ctypes.c_double()
        st = lib.silh_exact_noalloc(ctypes.byref(p), ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Ld.data_ptr()),
                                    None, *[ctypes.c_void_p(outs[key].data_ptr()) for key in "abs"],
                                    ctypes.byref(m))
        assert native.STATUS[st] == "SILH_OK", native.load_library().silh_last_error()
        return m.value

    torch.cuda.synchronize()
    m0 = call()
    free0 = torch.cuda.mem_get_info()[0]
    m1 = call()
    m2 = call()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0
    assert m0 == m1 == m2
    ref = native.silh_exact(Xd, Ld, 8, "eucl", "bf16")
    assert abs(m0 - ref["mean"]) <= S_ATOL


def test_noalloc_rejects_oversize_and_bad_labels():
    X, L = synth.tiny_case(3_000, 8, 4, seed=5)
    Xd, Ld = _dev(X, L)
    Lbad = Ld.clone()
    Lbad[17] = 4
    with pytest.raises(native.SilhError) as e:
        native.silh_exact_noalloc(Xd, Lbad, 4, "eucl", "fp32")
    assert e.value.name == "SILH_E_LABEL"
    Lone = torch.zeros_like(Ld)
    with pytest.raises(native.SilhError) as e:
        native.silh_exact_noalloc(Xd, Lone, 4, "eucl", "fp32")
    assert e.value.name == "SILH_E_K"
    # a valid call after the failed ones is unaffected
    ref = native.silh_exact(Xd, Ld, 4, "eucl", "fp32")
    got = native.silh_exact_noalloc(Xd, Ld, 4, "eucl", "fp32")
    _same(ref, got)
