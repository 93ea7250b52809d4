"""The C-ABI library loads, exports every symbol include/silh.h declares, and
rejects bad arguments before touching the GPU.  CPU only (no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2607_01993_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        with open(os.path.join(ROOT, "include", h)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(silh_[a-z_0-9]+)\s*\(", text))
    return names


def test_header_and_binding_agree():
    declared = _declared_symbols()
    assert declared == set(native.SIGNATURES), declared ^ set(native.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = native.load_library()
    for name in _declared_symbols():
        assert hasattr(lib, name), name
    assert lib.silh_version().decode().startswith("silh-mi355x")
    assert lib.silh_prof_count() > 0


def test_param_struct_layout():
    # offsets follow the C declaration order with natural alignment
    P = native.SilhParams
    assert P.n.offset == 0 and P.d.offset == 8 and P.k.offset == 12
    assert P.t.offset == 32 and P.eps.offset == 40 and P.seed.offset == 56
    assert ctypes.sizeof(P) == 88
    assert ctypes.sizeof(native.SilhSampleInfo) == 72


def _init(**kw):
    lib = native.load_library()
    base = dict(n=100, d=4, k=3, metric=0, prec=0, sampler=0, t=10, eps=0.0, delta=0.01, seed=1)
    base.update(kw)
    p = native._params(base["n"], base["d"], base["k"], base["metric"], base["prec"], base["sampler"],
                       base["t"], base["eps"], base["delta"], base["seed"], use_torch_alloc=False)
    for f in ("reserved0",):
        if f in kw:
            setattr(p, f, kw[f])
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    st = lib.silh_sample_init(ctypes.byref(p), fake, fake, None, ctypes.byref(out))
    return st, lib.silh_last_error().decode(), out


@pytest.mark.parametrize("kw,status", [
    (dict(n=1), 1), (dict(d=0), 1), (dict(d=257), 1), (dict(k=1), 1), (dict(k=5000), 1),
    (dict(metric=7), 1), (dict(prec=9), 1), (dict(sampler=3), 1), (dict(delta=0.0), 1),
    (dict(delta=1.0), 1), (dict(t=0, eps=0.0), 1), (dict(t=0, eps=1.5), 1),
    (dict(reserved0=1), 1), (dict(prec=1, metric=2), 7), (dict(prec=2, metric=3), 7), (dict(prec=1, metric=3), 7),
    (dict(prec=2, metric=0), 7), (dict(prec=2, metric=1, d=63), 7), (dict(prec=4), 1),
    (dict(d=300), 1),
])
def test_init_rejects_bad_params(kw, status):
    st, msg, out = _init(**kw)
    assert st == status, (st, msg)
    assert msg
    assert not out.value


def test_null_arguments():
    lib = native.load_library()
    assert lib.silh_sample_init(None, None, None, None, None) == 1
    assert lib.silh_pps_sample(None, None, None) == 1
    assert lib.silh_scores(None, None, None, None, None) == 1
    assert lib.silh_weighted_sums(None, None) == 1
    assert lib.silh_sample_view(None, None) == 1
    assert lib.silh_prof_enable(None, 1) == 1
    assert lib.silh_philox_uniform(0, -1, 5, 0, None, None) == 1
    assert lib.silh_philox_uniform(0, 0, 5, 0, None, None) == 1
    p = native._params(10, 4, 3, 0, 0, 0, 1, 0.0, 0.5, 0, use_torch_alloc=False)
    p.n = 1
    assert lib.silh_exact(ctypes.byref(p), ctypes.c_void_p(8), ctypes.c_void_p(8), None,
                          None, None, None, None) == 1
    assert lib.silh_coh_sep(None, None, None, None) == 1
    lib.silh_destroy(None)   # no-op


def test_rows_for_matches_the_hoeffding_size():
    """silh_rows_for is host arithmetic: compare it with the oracle's m and with
    the tail bound 2 exp(-m eps^2 / 2) <= delta that m is chosen for."""
    import math

    import oracle
    lib = native.load_library()
    for eps, delta in ((0.01, 0.01), (0.05, 0.1), (0.2, 0.5), (0.5, 0.01), (0.003, 0.05)):
        m = ctypes.c_int64()
        assert lib.silh_rows_for(eps, delta, ctypes.byref(m)) == 0
        assert m.value == oracle.m_for(eps, delta)
        assert 2.0 * math.exp(-m.value * eps * eps / 2.0) <= delta * (1 + 1e-12)
        assert 2.0 * math.exp(-(m.value - 1) * eps * eps / 2.0) > delta
    m = ctypes.c_int64()
    for eps, delta in ((0.0, 0.1), (1.0, 0.1), (0.1, 0.0), (0.1, 1.0), (1e-6, 0.01)):
        assert lib.silh_rows_for(eps, delta, ctypes.byref(m)) == 1, (eps, delta)
    assert lib.silh_rows_for(0.1, 0.1, None) == 1


def test_rows_calls_reject_bad_arguments():
    lib = native.load_library()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    assert lib.silh_draw_rows(1, 0, 5, fake, None) == 1          # n < 1
    assert lib.silh_draw_rows(1, 1 << 31, 5, fake, None) == 1    # n > 2^30
    assert lib.silh_draw_rows(1, 10, -1, fake, None) == 1        # m < 0
    assert lib.silh_draw_rows(1, 10, 5, None, None) == 1         # rows NULL
    assert lib.silh_scores_rows(None, fake, 5, None, None, None, None) == 1
    p = native._params(10, 4, 3, 0, 0, 0, 1, 0.0, 0.5, 0, use_torch_alloc=False)
    p.k = 1
    assert lib.silh_exact_rows(ctypes.byref(p), fake, fake, fake, 5, None, None, None, None, None) == 1


def test_server_layouts_and_argument_checks():
    P = native
    assert ctypes.sizeof(P.SilhServerCfg) == 16
    assert ctypes.sizeof(P.SilhRequest) == 64 and P.SilhRequest.t.offset == 32 and P.SilhRequest.m.offset == 56
    assert ctypes.sizeof(P.SilhResult) == 48 + 160
    lib = native.load_library()
    out = ctypes.c_void_p()
    for w, r, b in ((0, 0, 1 << 30), (65, 0, 1 << 30), (2, 2, 1 << 30), (2, -1, 1 << 30), (2, 0, 0)):
        cfg = P.SilhServerCfg(w, r, b)
        assert lib.silh_server_create(ctypes.byref(cfg), ctypes.byref(out)) == 1
        assert not out.value
    assert lib.silh_server_create(None, ctypes.byref(out)) == 1
    assert lib.silh_server_submit(None, None, None) == 1
    assert lib.silh_server_wait(None, 1, None) == 1
    assert lib.silh_server_drain(None) == 1
    assert lib.silh_server_add_dataset(None, None, 10, 4, None) == 1
    lib.silh_server_destroy(None)
    assert lib.silh_server_launches(None) == -1
    t0 = lib.silh_server_now_ns()
    assert lib.silh_server_now_ns() >= t0 > 0


def test_graph_layout_and_argument_checks():
    assert ctypes.sizeof(native.SilhGraphInfo) == 32
    lib = native.load_library()
    out = ctypes.c_void_p()
    p = native._params(1000, 8, 2, "eucl", "bf16", "pps", 32, 0.0, 0.01, 1, use_torch_alloc=False)
    fake = ctypes.c_void_p(256)  # never dereferenced: every check below fails first
    ks = (ctypes.c_int32 * 2)(3, 4)
    assert lib.silh_graph_create(None, fake, fake, ks, 2, 2, 0.0, None, ctypes.byref(out)) == 1
    assert lib.silh_graph_create(ctypes.byref(p), fake, fake, ks, 0, 2, 0.0, None, ctypes.byref(out)) == 1
    for chains in (0, 17):
        assert lib.silh_graph_create(ctypes.byref(p), fake, fake, ks, 2, chains, 0.0, None, ctypes.byref(out)) == 1
    bad = (ctypes.c_int32 * 2)(3, 1)  # k = 1 for the second clustering
    assert lib.silh_graph_create(ctypes.byref(p), fake, fake, bad, 2, 2, 0.0, None, ctypes.byref(out)) == 1
    assert not out.value
    assert lib.silh_graph_run(None, None, None, None, None, None) == 1
    assert lib.silh_graph_get_info(None, None) == 1
    shape, S = ctypes.c_int32(), ctypes.c_int64()
    assert lib.silh_graph_choice(None, 0, ctypes.byref(shape), ctypes.byref(S)) == 1
    lib.silh_graph_destroy(None)


def test_exact_noalloc_argument_checks():
    """silh_exact_noalloc checks its arguments and the size of its static
    scratch array before it touches the device."""
    lib = native.load_library()
    p = native._params(10, 4, 3, 0, 0, 0, 1, 0.0, 0.5, 0, use_torch_alloc=False)
    p.n = 1
    assert lib.silh_exact_noalloc(ctypes.byref(p), ctypes.c_void_p(8), ctypes.c_void_p(8), None,
                                  None, None, None, None) == 1
    p = native._params(4_000_000, 32, 16, "eucl", "bf16", "pps", 1, 0.0, 0.5, 0, use_torch_alloc=False)
    assert lib.silh_exact_noalloc(ctypes.byref(p), ctypes.c_void_p(8), ctypes.c_void_p(8), None,
                                  None, None, None, None) == 1
    assert b"scratch" in lib.silh_last_error()
    p = native._params(1000, 32, 16, "eucl", "bf16", "pps", 1, 0.0, 0.5, 0, use_torch_alloc=False)
    assert lib.silh_exact_noalloc(ctypes.byref(p), None, ctypes.c_void_p(8), None, None, None, None, None) == 1
