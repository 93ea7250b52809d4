"""The four distance functions of the paper's experiments (Section 5.1.2),
evaluated in float64 on float32 inputs (the promotion is exact).

TEST INFRASTRUCTURE ONLY: part of the CPU oracle.

The method treats d(.,.) as a black box (Section 2; Section 4.1.1); only its
values enter.  Every function here accumulates over coordinates in increasing
coordinate order, one rounding per elementary operation (no fused
multiply-add), so that the result is a fixed, reproducible function of the
inputs.

* Euclidean  d(x,y) = sqrt(sum_i (x_i - y_i)^2)             (Section 2, footnote; Section 5.1.2)
* Manhattan  d(x,y) = sum_i |x_i - y_i|                      (Section 5.1.2)
* Canberra   d(x,y) = sum_i |x_i - y_i| / (|x_i| + |y_i|)    (Section 5.1.2);
  a coordinate with |x_i| + |y_i| = 0 contributes 0 (reading: 0/0 -> 0).
* Cosine     the printed formula is garbled (its numerator reads as a sum of
  coordinate differences).  Reading: d(x,y) = 1 - x.y / (|x| |y|), with the
  similarity taken as 0 when either norm is 0, and the result clamped to
  [0, 2].
"""
from __future__ import annotations

import numpy as np

EUCL, COS, MANH, CANB = 0, 1, 2, 3
NAMES = {"eucl": EUCL, "cos": COS, "manh": MANH, "canb": CANB}


def metric_id(metric) -> int:
    return NAMES[metric] if isinstance(metric, str) else int(metric)


def dist_matrix(A: np.ndarray, B: np.ndarray, metric) -> np.ndarray:
    """All pairwise distances between the rows of A (m x z) and B (q x z),
    as an (m, q) float64 array."""
    metric = metric_id(metric)
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, z = A.shape
    q = B.shape[0]
    if metric == EUCL:
        acc = np.zeros((m, q))
        for c in range(z):
            diff = A[:, c][:, None] - B[:, c][None, :]
            acc = acc + diff * diff
        return np.sqrt(acc)
    if metric == MANH:
        acc = np.zeros((m, q))
        for c in range(z):
            acc = acc + np.abs(A[:, c][:, None] - B[:, c][None, :])
        return acc
    if metric == CANB:
        acc = np.zeros((m, q))
        for c in range(z):
            num = np.abs(A[:, c][:, None] - B[:, c][None, :])
            den = np.abs(A[:, c])[:, None] + np.abs(B[:, c])[None, :]
            term = np.divide(num, den, out=np.zeros_like(num), where=den > 0)
            acc = acc + term
        return acc
    if metric == COS:
        dot = np.zeros((m, q))
        na = np.zeros(m)
        nb = np.zeros(q)
        for c in range(z):
            dot = dot + A[:, c][:, None] * B[:, c][None, :]
            na = na + A[:, c] * A[:, c]
            nb = nb + B[:, c] * B[:, c]
        den = np.sqrt(na)[:, None] * np.sqrt(nb)[None, :]
        sim = np.divide(dot, den, out=np.zeros_like(dot), where=den > 0)
        return np.clip(1.0 - sim, 0.0, 2.0)
    raise ValueError(f"unknown metric {metric}")


def dist_to_point(A: np.ndarray, y: np.ndarray, metric) -> np.ndarray:
    """Distances from every row of A to the single point y, shape (m,)."""
    return dist_matrix(A, np.asarray(y)[None, :], metric)[:, 0]
