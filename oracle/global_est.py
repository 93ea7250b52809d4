"""Subsampled estimators of the silhouette of a clustering (Section 4.2):
gl-s (Eq. 8) and gl-pps-s / gl-uni-s (Eq. 10), float64.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see the package header).

* gl-s: the mean of the exact silhouette s(e) over m elements drawn uniformly
  at random from V (Eq. 8); Theorem 4 asks for m >= (2/eps^2) ln(2/delta).
* gl-pps-s: Phase 1 of Algorithm 1 fixes every s_hat(e); the estimate is the
  mean of s_hat over m indices drawn uniformly at random from {1..n}
  (Eq. 10), m >= (2/eps_2^2) ln(2/delta_2) by the lemma after it.  gl-uni-s is
  the same with the uniform sampler (Section 4.1.3) in Phase 1.

Readings: the m elements are drawn independently, with replacement (the
Hoeffding argument of both bounds needs independent draws; the text only
says "uniformly at random").  Draw i is the integer floor(B_i * n / 2^53),
B_i the 53-bit integer of the Philox draw for counter i in the row stream,
which is uniform on {0..n-1} up to a bias below n / 2^53.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import STREAM_ROWS, bits53
from .silhouette import estimate, exact, global_mean, sample


def m_for(eps: float, delta: float) -> int:
    """Sample size of Theorem 4 / the lemma after Eq. 10: ceil((2/eps^2) ln(2/delta))."""
    if not (0.0 < eps < 1.0 and 0.0 < delta < 1.0):
        raise ValueError("eps and delta must lie in (0, 1)")
    return int(math.ceil((2.0 / (eps * eps)) * math.log(2.0 / delta)))


def draw_rows(seed: int, n: int, m: int) -> np.ndarray:
    """m indices in [0, n), independent and uniform, with replacement."""
    b = bits53(seed, np.arange(m, dtype=np.uint64), STREAM_ROWS)
    return np.array([(int(v) * int(n)) >> 53 for v in b], dtype=np.int64)


def subset_mean(values) -> float:
    """(1/m) sum over the m drawn entries (duplicates counted each time)."""
    return global_mean(values)


def gl_s(X, labels, k: int, metric, m: int, seed: int) -> dict:
    """Eq. 8: the mean of the exact s(e) over m uniform draws."""
    rows = draw_rows(seed, np.asarray(X).shape[0], m)
    ex = exact(X, labels, k, metric, rows=rows)
    ex["mean"] = subset_mean(ex["s"])
    return ex


def gl_pps_s(X, labels, k: int, metric, t: int, delta: float, seed: int, m: int, rows_seed: int,
             sampler: str = "pps") -> dict:
    """Eq. 10: Phase 1 (PPS, or uniform for gl-uni-s), then the mean of
    s_hat over m uniform draws of rows."""
    smp = sample(X, labels, k, metric, t, delta, seed, sampler)
    rows = draw_rows(rows_seed, np.asarray(X).shape[0], m)
    est = estimate(X, labels, k, metric, smp, rows=rows)
    est["mean"] = subset_mean(est["s"])
    est["sample"] = smp
    return est


def sweep(X, label_sets, ks, metric, t: int, delta: float, seed: int, m: int = 0, sampler: str = "pps") -> dict:
    """The choice of k by the global silhouette (Section 5, selection of the
    best value of k): for each clustering, s_hat_2 (Eq. 9) or, with m > 0,
    the Eq. 10 mean over m row draws (row seed = seed); the index of the
    largest (the first among equal ones)."""
    means = []
    n = np.asarray(X).shape[0]
    for L, k in zip(label_sets, ks):
        smp = sample(X, L, k, metric, t, delta, seed, sampler)
        if m > 0:
            est = estimate(X, L, k, metric, smp, rows=draw_rows(seed, n, m))
            means.append(subset_mean(est["s"]))
        else:
            means.append(estimate(X, L, k, metric, smp)["mean"])
    means = np.array(means)
    return {"means": means, "best": int(np.argmax(means))}
