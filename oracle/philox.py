"""Philox4x32-10 counter-based generator, written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",
SC'11, Section 4: the Philox S-box with two 32x32->64 multiplies per round and
a Weyl-sequence key schedule).

TEST INFRASTRUCTURE ONLY: this is part of the CPU oracle.

The paper's Poisson sampling (Algorithm 1, the draws of the initial sample and
of the final sample, and the uniform variant of Section 4.1.3) needs one
independent uniform per element and per draw; the paper does not say how they
are produced.  Reading used here: the uniform for element `gid` in draw
`stream` is built from Philox4x32-10 with key (seed_lo, seed_hi) and counter
(gid_lo, gid_hi, stream, 0), taking the first two 32-bit output words w0, w1
as U = (w0 * 2^21 + floor(w1 / 2^11)) * 2^-53, a double in [0, 1).
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# round multipliers and key increments of Philox4x32 (SC'11, Table 2 / text)
M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)

STREAM_F0 = 0   # initial sample F^0 (Algorithm 1, Phase 1, Poisson draw with fixed rate)
STREAM_PPS = 1  # final PPS sample F (Algorithm 1, Poisson draw with rates p_e)
STREAM_UNI = 2  # uniform Poisson sample (Section 4.1.3)
STREAM_ROWS = 3  # the m row indices of the subsampled global estimators (Section 4.2)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (or scalars) of uint32 values, key: 2 of them.
    Returns 4 uint64 arrays holding the 32-bit output words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & MASK32 for k in key)
    for r in range(10):
        p0 = M0 * c0            # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
        if r != 9:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
    return c0, c1, c2, c3


def bits53(seed: int, gid, stream: int) -> np.ndarray:
    """The 53-bit integer w0 * 2^21 + floor(w1 / 2^11) behind U(seed, gid,
    stream), as uint64, vectorised over gid."""
    gid = np.asarray(gid, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32))
    ctr = (gid & MASK32, gid >> np.uint64(32), np.full(gid.shape, stream, dtype=np.uint64),
           np.zeros(gid.shape, dtype=np.uint64))
    w0, w1, _, _ = philox4x32_10(ctr, key)
    return (w0 << np.uint64(21)) | (w1 >> np.uint64(11))


def uniform53(seed: int, gid, stream: int) -> np.ndarray:
    """U(seed, gid, stream) in [0, 1) as float64, vectorised over gid."""
    return bits53(seed, gid, stream).astype(np.float64) * (2.0 ** -53)
