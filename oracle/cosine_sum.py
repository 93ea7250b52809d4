"""W_hat of Algorithm 1, Phase 2, for the cosine distance through its linear
form, float64.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see the package header).

With the reading of the garbled printed formula used throughout the oracle
(Section 5.1.2: d(x, y) = 1 - x.y / (|x| |y|), similarity 0 for a zero
vector), the distance is affine in the unit vector y/|y|:

    W_hat_{C_j}(e) = sum_{y in F_j} w_y (1 - x_hat . y_hat)
                   = T_j - x_hat . Z_j,
    T_j = sum_{y in F_j} w_y,   Z_j = sum_{y in F_j, y != 0} w_y y_hat,

with w = 1/p and x_hat = 0 for a zero row (its distance to everything is 1).
This is the same sum as `silhouette.estimate` evaluates pair by pair, in
O(n k d) instead of O(n |F| d) operations, which makes the estimator's value
at millions of rows computable on a CPU.  The clamp of d to [0, 2] is dropped:
1 - x_hat . y_hat lies in [0, 2] up to float64 rounding, so the two forms
differ by rounding only (the pin test holds them to 1e-9).
"""
from __future__ import annotations

import numpy as np

from .silhouette import global_mean, scores_from_weights


def _unit_rows(A):
    A = np.asarray(A, dtype=np.float64)
    nrm = np.sqrt((A * A).sum(axis=1))
    out = np.zeros_like(A)
    nz = nrm > 0
    out[nz] = A[nz] / nrm[nz, None]
    return out


def cosine_weights(X, k: int, smp: dict, rows=None, block: int = 1 << 16):
    """W_hat (len(rows) x k) for the cosine distance, Phase 2 of Algorithm 1,
    by the linear form above; `smp` is the result of `silhouette.sample`."""
    X = np.asarray(X)
    p = smp["p"]
    T = np.zeros(k)
    Z = np.zeros((k, X.shape[1]))
    for j in range(k):
        F = smp["F"][j]
        if F.shape[0] == 0:
            continue
        w = 1.0 / p[F]
        T[j] = w.sum()
        Z[j] = (w[:, None] * _unit_rows(X[F])).sum(axis=0)
    idx = np.arange(X.shape[0]) if rows is None else np.asarray(rows)
    W = np.empty((idx.shape[0], k))
    for r0 in range(0, idx.shape[0], block):
        xh = _unit_rows(X[idx[r0:r0 + block]])
        W[r0:r0 + xh.shape[0]] = T[None, :] - xh @ Z.T
    return W


def cosine_estimate(X, labels, k: int, smp: dict, rows=None):
    """a_hat, b_hat, s_hat (Eq. 5) from `cosine_weights`, and the Eq. 9 mean
    when all rows are evaluated."""
    labels = np.asarray(labels)
    idx = np.arange(np.asarray(X).shape[0]) if rows is None else np.asarray(rows)
    W = cosine_weights(X, k, smp, rows=idx)
    a, b, s = scores_from_weights(W, labels[idx], smp["sizes"])
    out = {"W": W, "a": a, "b": b, "s": s, "rows": idx}
    if rows is None:
        out["mean"] = global_mean(s)
    return out
