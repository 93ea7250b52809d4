"""Device memory without allocator hooks: the library's per-(device, stream)
block cache.  Requests give the same results bit for bit as with PyTorch's
caching allocator, on the default stream and on a second stream, and
repeated requests reuse the cached blocks instead of taking more memory."""
import numpy as np
import pytest
import torch

from paper_2607_01993_amd import native, synth

pytestmark = pytest.mark.gpu


def _request(Xd, Ld, k, prec, torch_alloc, stream=None):
    ctx = native.silh_sample_init(Xd, Ld, k, "eucl", prec, t=48, seed=5, stream=stream,
                                  use_torch_alloc=torch_alloc)
    native.silh_pps_sample(ctx)
    res = native.silh_scores(ctx)
    native.silh_destroy(ctx)
    return res


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_block_cache_matches_torch_allocator(prec):
    X, L = synth.tiny_case(20000, 16, 6, seed=51)
    Xd, Ld = torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda()
    ref = _request(Xd, Ld, 6, prec, True)
    got = _request(Xd, Ld, 6, prec, False)
    assert got["mean"] == ref["mean"]
    for key in ("a", "b", "s"):
        assert torch.equal(got[key], ref[key]), key
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        other = _request(Xd, Ld, 6, prec, False, stream=side)
    side.synchronize()
    assert other["mean"] == ref["mean"]
    assert torch.equal(other["s"], ref["s"])


def test_block_cache_reuses_blocks():
    X, L = synth.tiny_case(200000, 32, 8, seed=52)
    Xd, Ld = torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda()
    first = _request(Xd, Ld, 8, "bf16", False)["mean"]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    means = [_request(Xd, Ld, 8, "bf16", False)["mean"] for _ in range(10)]
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert np.all(np.array(means) == first)
    # the outputs a, b, s are PyTorch tensors freed to its cache; the
    # library's own buffers (tens of MB per request here) come back from the
    # block cache, so ten more requests take no further device memory
    assert free0 - free1 < 8 << 20, (free0, free1)
