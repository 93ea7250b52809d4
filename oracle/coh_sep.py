"""Cohesion and separation of a clustering (Appendix B), float64.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see the package header).

Coh = (1/2) sum_j sum_{e in C_j} W_{C_j}(e) / sum_j C(|C_j|, 2): the mean
distance over unordered pairs inside clusters; Sep = sum_{j1 < j2} sum_{e in
C_j1} W_{C_j2}(e) / sum_{j1 < j2} |C_j1| |C_j2|: the mean distance over pairs
in different clusters.  The estimates put W_hat (Algorithm 1, Phase 2) in
place of W.  Reading: the separation denominator printed with |C_{j-1}| is
|C_j1| |C_j2| (the form the appendix's own rewriting uses).
"""
from __future__ import annotations

import math

import numpy as np


def coh_sep_from_weights(W, labels, sizes):
    """Coh and Sep from per-element cluster sums W (n x k) and cluster sizes."""
    W = np.asarray(W, dtype=np.float64)
    labels = np.asarray(labels)
    sizes = np.asarray(sizes, dtype=np.int64)
    n, k = W.shape
    own = W[np.arange(n), labels]
    coh_num = 0.5 * math.fsum(own.tolist())
    coh_den = float(sum(int(c) * (int(c) - 1) // 2 for c in sizes))
    later = np.arange(k)[None, :] > labels[:, None]          # j2 > own cluster
    sep_num = math.fsum(W[later].tolist())
    tot = int(sizes.sum())
    sep_den = float(sum(int(sizes[j]) * (tot - int(sizes[: j + 1].sum())) for j in range(k)))
    return {"coh": coh_num / coh_den if coh_den > 0 else 0.0,
            "sep": sep_num / sep_den if sep_den > 0 else 0.0,
            "coh_num": coh_num, "coh_den": coh_den, "sep_num": sep_num, "sep_den": sep_den}
