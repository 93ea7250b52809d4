"""The serving runtime (include/silh_server.h) on the GPU: results of requests
run concurrently by the server equal those of the same requests run alone
through silh.h; admission, argument checks and per-request failures."""
import math

import numpy as np
import pytest
import torch

from paper_2607_01993_amd import native, synth

pytestmark = pytest.mark.gpu


def _direct(X, L, k, metric, prec, sampler, t, seed):
    ctx = native.silh_sample_init(X, L, k, metric, prec, sampler, t=t, delta=0.01, seed=seed)
    S, _ = native.silh_pps_sample(ctx)
    mean = native.silh_scores(ctx, a=False, b=False, s=False, mean=True)["mean"]
    native.silh_destroy(ctx)
    return S, mean


def _datasets():
    X1, L1 = synth.tiny_case(6000, 8, 5, seed=61)
    X2, L2 = synth.vmf_blobs(5000, 64, 6, seed=62, kappa=40.0)
    X3, L3 = synth.tiny_case(4000, 16, 4, seed=63)
    return [(torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda(), k)
            for X, L, k in ((X1, L1, 5), (X2, L2, 6), (X3, L3, 4))]


REQS = [  # (dataset, metric, prec, sampler, t, seed)
    (0, "eucl", "bf16", "pps", 64, 1), (1, "cos", "fp8", "pps", 128, 2), (2, "manh", "fp32", "pps", 32, 3),
    (0, "canb", "fp32", "uni", 48, 4), (1, "cos", "bf16", "pps", 256, 5), (2, "eucl", "fp32", "pps", 1024, 6),
    (0, "eucl", "fp32_valu", "pps", 64, 7), (1, "eucl", "bf16", "uni", 64, 8), (2, "cos", "fp32", "pps", 16, 9),
    (0, "manh", "fp32", "pps", 256, 10), (1, "canb", "fp32", "pps", 64, 11), (2, "eucl", "bf16", "pps", 64, 12),
]


@pytest.mark.parametrize("workers", [1, 3])
def test_server_results_equal_direct_calls(workers):
    ds = _datasets()
    srv = native.Server(workers=workers, hbm_budget_bytes=8 << 30)
    ids = [srv.add_dataset(X) for X, _, _ in ds]
    tickets = []
    for (di, metric, prec, sampler, t, seed) in REQS:
        X, L, k = ds[di]
        tickets.append(srv.submit(ids[di], L, k, metric, prec, sampler, t=t, seed=seed))
    results = [srv.wait(tk) for tk in tickets]
    srv.close()
    for (di, metric, prec, sampler, t, seed), res in zip(REQS, results):
        X, L, k = ds[di]
        assert res["status"] == "SILH_OK", res
        S, mean = _direct(X, L, k, metric, prec, sampler, t, seed)
        assert res["S"] == S
        assert res["s_mean"] == mean, (metric, prec, res["s_mean"], mean)
        assert res["submit_ns"] <= res["start_ns"] <= res["done_ns"]


def test_server_admission_under_a_small_budget():
    """A budget that fits one request at a time: requests still all finish,
    and never more than one runs at once (start after the previous done)."""
    ds = _datasets()
    X, L, k = ds[0]
    # the estimate of one such request is 24 n + the distances kept between
    # the W pass and the draw (their capacity, n (2.5 ln(5k/delta) + 8)
    # doubles) + (a few KB of sample) + 1 MiB: 1.5 times its main part fits
    # one request, never two
    n = X.shape[0]
    kept = 8 * int(min(n * (2.5 * math.log(5.0 * k / 0.01) + 8.0), 2 ** 27))
    srv = native.Server(workers=4, hbm_budget_bytes=int(1.5 * (24 * n + kept + (1 << 20))))
    did = srv.add_dataset(X)
    tks = [srv.submit(did, L, k, "eucl", "bf16", t=32, seed=s) for s in range(6)]
    res = [srv.wait(tk) for tk in tks]
    srv.close()
    assert all(r["status"] == "SILH_OK" for r in res)
    spans = sorted((r["start_ns"], r["done_ns"]) for r in res)
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        assert s1 >= e0
    # a request whose estimate alone exceeds the budget is refused at submit
    srv = native.Server(workers=1, hbm_budget_bytes=1 << 20)
    did = srv.add_dataset(X)
    with pytest.raises(native.SilhError) as e:
        srv.submit(did, L, k, "eucl", "bf16", t=32)
    assert e.value.name == "SILH_E_NOMEM"
    srv.close()


def test_server_checks_requests_and_reports_failures():
    ds = _datasets()
    X, L, k = ds[0]
    srv = native.Server(workers=2, hbm_budget_bytes=4 << 30)
    did = srv.add_dataset(X)
    for kw, name in ((dict(dataset=did + 7), "SILH_E_ARG"), (dict(k=1), "SILH_E_ARG"),
                     (dict(prec="fp8"), "SILH_E_UNSUPPORTED"), (dict(t=0), "SILH_E_ARG")):
        args = dict(dataset=did, k=k, metric="eucl", prec="bf16", t=32)
        args.update(kw)
        with pytest.raises(native.SilhError) as e:
            srv.submit(args.pop("dataset"), L, **args)
        assert e.value.name == name, (kw, e.value.name)
    bad = L.clone()
    bad[17] = k                     # a label outside [0, k): found by the worker
    tb = srv.submit(did, bad, k, "eucl", "bf16", t=32)
    tg = srv.submit(did, L, k, "eucl", "bf16", t=32)
    rb, rg = srv.wait(tb), srv.wait(tg)
    assert rb["status"] == "SILH_E_LABEL" and "label" in rb["message"]
    assert rg["status"] == "SILH_OK"
    with pytest.raises(native.SilhError):
        srv.wait(tb)                # retired
    srv.drain()
    srv.close()
