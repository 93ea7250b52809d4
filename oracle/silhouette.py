"""Plain float64 CPU oracle for the exact silhouette and for the PPS / uniform
sampled silhouette estimator of "Scalable and Distributed Silhouette
Approximation" (arxiv 2607.01993).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark use this package; the product path never imports it.  It
shares no code with the HIP path: the only thing both sides see is the seeded
input arrays.

What is computed, and where the paper defines it:

* exact silhouette: a(e), b(e), s(e) (Section 2, Eqs. 1-2), s(e) = 0 for a
  singleton cluster (Section 2, text after Eq. 2), s(C) = mean (Eq. 3);
* W_{C_j}(e) = sum of distances to cluster C_j (Section 4.1.1, Eq. 4), with
  a = W_C/(|C|-1) and b = min_{j != C} W_{C_j}/|C_j|;
* Phase 1 of Algorithm 1 (PPS sampling): per cluster with |C_j| > t, an
  initial Poisson sample F^0 with rate (2/|C_j|) ln(5k/delta), the weights
  W(e_bar) of its members, gamma_e = max{1/|C_j|, max d(e,e_bar)/W(e_bar)},
  p_e = min{1, t gamma_e}, then the Poisson sample F with rates p_e; clusters
  with |C_j| <= t are taken whole (p = 1);
* the uniform variant (Section 4.1.3): rate t/|C_j| for every element;
* Phase 2 of Algorithm 1: W_hat_{C_j}(e) = sum_{e' in F_j} d(e,e')/p_{e'},
  a_hat, b_hat, s_hat as above (Eq. 5);
* the global estimate s_hat_2 = mean of s_hat (Section 4.2, Eq. 9).

Readings taken where the paper is silent or inconsistent:

* t: the experiments set t directly (Section 5.1.3); when it is derived from
  eps it uses the form of Lemma 1, t = ceil((3c/eps^2) ln(5nk/delta)), c = 18
  (Algorithm 1 prints c eps^-2 ln(5nk/delta) instead).
* the initial-sample rate is clamped to at most 1; the k in ln(5k/delta) is the
  number of clusters passed in, empty ones included.
* an empty initial sample gives gamma_e = 1/|C_j| (the inner max over an empty
  set is dropped); an initial element with W(e_bar) = 0 is skipped.
* a_hat of a singleton is 0 and its s_hat is 0 (Lemma 2's proof); s_hat = 0
  whenever max(a_hat, b_hat) = 0; empty clusters are skipped in the min.
* the random numbers come from oracle.philox (counter = element id, stream).
"""
from __future__ import annotations

import math

import numpy as np

from .distance import dist_matrix, metric_id
from .philox import STREAM_F0, STREAM_PPS, STREAM_UNI, uniform53

C_LEMMA1 = 18.0


def default_t(eps: float, delta: float, n: int, k: int) -> int:
    """Sample-size parameter of Lemma 1: ceil((3c/eps^2) ln(5nk/delta)), c = 18."""
    return int(math.ceil((3.0 * C_LEMMA1 / (eps * eps)) * math.log(5.0 * n * k / delta)))


def cluster_members(labels: np.ndarray, k: int):
    """Ids of the elements of each cluster, ascending."""
    labels = np.asarray(labels)
    order = np.argsort(labels, kind="stable")
    sizes = np.bincount(labels, minlength=k)
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    return [order[bounds[j]:bounds[j + 1]] for j in range(k)], sizes.astype(np.int64)


def scores_from_weights(W: np.ndarray, own: np.ndarray, sizes: np.ndarray):
    """a, b, s from per-cluster distance sums W (rows x k) (Section 4.1.1, Eq. 4
    reformulation; Eq. 1 / Eq. 5 for s)."""
    W = np.asarray(W, dtype=np.float64)
    own = np.asarray(own)
    sizes = np.asarray(sizes, dtype=np.int64)
    rows = np.arange(W.shape[0])
    cown = sizes[own]
    a = np.zeros(W.shape[0])
    multi = cown > 1
    a[multi] = W[rows[multi], own[multi]] / (cown[multi] - 1).astype(np.float64)
    safe = np.where(sizes > 0, sizes, 1).astype(np.float64)
    cand = W / safe[None, :]
    cand[:, sizes == 0] = np.inf
    cand[rows, own] = np.inf
    b = cand.min(axis=1)
    M = np.maximum(a, b)
    s = np.zeros(W.shape[0])
    ok = multi & (M > 0)
    s[ok] = (b[ok] - a[ok]) / M[ok]
    return a, b, s


def global_mean(s) -> float:
    """Eq. 3 / Eq. 9: (1/n) * sum, the sum exactly rounded."""
    s = np.asarray(s, dtype=np.float64)
    return math.fsum(s.tolist()) / s.shape[0]


def exact(X, labels, k: int, metric, rows=None, block: int = 512):
    """Exact silhouette (Eqs. 1-3) for `rows` (all rows by default).

    Returns dict with W (rows x k), a, b, s and, when all rows are evaluated,
    the mean s(C)."""
    X = np.asarray(X)
    labels = np.asarray(labels)
    members, sizes = cluster_members(labels, k)
    if np.count_nonzero(sizes) < 2:
        raise ValueError("fewer than two nonempty clusters")
    idx = np.arange(X.shape[0]) if rows is None else np.asarray(rows)
    W = np.zeros((idx.shape[0], k))
    for r0 in range(0, idx.shape[0], block):
        r = idx[r0:r0 + block]
        for j in range(k):
            if sizes[j] == 0:
                continue
            D = dist_matrix(X[r], X[members[j]], metric)
            W[r0:r0 + r.shape[0], j] = D.sum(axis=1)
    a, b, s = scores_from_weights(W, labels[idx], sizes)
    out = {"W": W, "a": a, "b": b, "s": s, "rows": idx, "sizes": sizes}
    if rows is None:
        out["mean"] = global_mean(s)
    return out


def sample(X, labels, k: int, metric, t: int, delta: float, seed: int, sampler: str = "pps"):
    """Phase 1 of Algorithm 1 (PPS), or the uniform Poisson sampler of
    Section 4.1.3 (sampler="uni").

    Returns a dict with, per cluster j: F[j] (sampled ids, ascending), F0[j]
    and W0[j] (initial sample and its weights, PPS only), q[j] (initial rate);
    and per element: p (inclusion probability; 1 for clusters taken whole) and
    gamma (NaN where not defined)."""
    X = np.asarray(X)
    labels = np.asarray(labels)
    n = X.shape[0]
    members, sizes = cluster_members(labels, k)
    p = np.ones(n)
    gamma = np.full(n, np.nan)
    F, F0, W0, q = [], [], [], np.zeros(k)
    lnterm = math.log(5.0 * k / delta)
    for j in range(k):
        idx = members[j]
        m = idx.shape[0]
        if m <= t:                      # Algorithm 1: small cluster taken whole
            F.append(idx.copy())
            F0.append(idx[:0].copy())
            W0.append(np.zeros(0))
            continue
        if sampler == "uni":            # Section 4.1.3: rate t/|C_j| for every element
            pj = min(1.0, float(t) / float(m))
            p[idx] = pj
            u = uniform53(seed, idx, STREAM_UNI)
            F.append(idx[u < pj])
            F0.append(idx[:0].copy())
            W0.append(np.zeros(0))
            continue
        # initial Poisson sample with rate (2/|C_j|) ln(5k/delta), clamped to 1
        qj = min(1.0, (2.0 / float(m)) * lnterm)
        q[j] = qj
        u0 = uniform53(seed, idx, STREAM_F0)
        f0 = idx[u0 < qj]
        # W(e_bar): sum of distances from e_bar to all of C_j
        D = dist_matrix(X[idx], X[f0], metric)            # (m, |F0|)
        w0 = np.array([math.fsum(D[:, c].tolist()) for c in range(f0.shape[0])])
        # gamma_e = max{1/|C_j|, max over e_bar with W(e_bar) > 0 of d(e,e_bar)/W(e_bar)}
        g = np.full(m, 1.0 / float(m))
        pos = w0 > 0
        if np.any(pos):
            ratio = D[:, pos] / w0[pos][None, :]
            g = np.maximum(g, ratio.max(axis=1))
        gamma[idx] = g
        pe = np.minimum(1.0, float(t) * g)
        p[idx] = pe
        u1 = uniform53(seed, idx, STREAM_PPS)
        F.append(idx[u1 < pe])
        F0.append(f0)
        W0.append(w0)
    return {"F": F, "F0": F0, "W0": W0, "q": q, "p": p, "gamma": gamma, "sizes": sizes,
            "members": members, "t": t, "sampler": sampler}


def estimate(X, labels, k: int, metric, smp: dict, rows=None, block: int = 512):
    """Phase 2 of Algorithm 1: W_hat_{C_j}(e) = sum_{e' in F_j} d(e,e')/p_{e'}
    and a_hat, b_hat, s_hat for `rows` (all rows by default); the mean (Eq. 9)
    when all rows are evaluated."""
    X = np.asarray(X)
    labels = np.asarray(labels)
    sizes = smp["sizes"]
    if np.count_nonzero(sizes) < 2:
        raise ValueError("fewer than two nonempty clusters")
    idx = np.arange(X.shape[0]) if rows is None else np.asarray(rows)
    p = smp["p"]
    What = np.zeros((idx.shape[0], k))
    for r0 in range(0, idx.shape[0], block):
        r = idx[r0:r0 + block]
        for j in range(k):
            Fj = smp["F"][j]
            if Fj.shape[0] == 0:
                continue
            D = dist_matrix(X[r], X[Fj], metric)
            What[r0:r0 + r.shape[0], j] = (D / p[Fj][None, :]).sum(axis=1)
    a, b, s = scores_from_weights(What, labels[idx], sizes)
    out = {"W": What, "a": a, "b": b, "s": s, "rows": idx}
    if rows is None:
        out["mean"] = global_mean(s)
    return out


def pps_silhouette(X, labels, k: int, metric, t: int, delta: float = 0.01, seed: int = 0,
                   sampler: str = "pps", rows=None):
    """Algorithm 1 end to end (Phase 1 then Phase 2), plus the Eq. 9 mean."""
    smp = sample(X, labels, k, metric, t, delta, seed, sampler)
    est = estimate(X, labels, k, metric, smp, rows=rows)
    est["sample"] = smp
    return est
