"""Philox4x32-10 counter-based generator, written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC 2011, section on the Philox S-box/P-box construction).

TEST INFRASTRUCTURE: part of the CPU oracle.  The GPU library carries its own,
separately written generator; the two meet only through the published
definition and the known-answer vectors in ``tests/golden``.

Definition used here (4 words of 32 bits, 2 key words, 10 rounds):

* one round maps counter (x0, x1, x2, x3) under key (k0, k1) to
  ``(hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0))``
  with multipliers M0 = 0xD2511F53, M1 = 0xCD9E8D57;
* between rounds the key is bumped by the Weyl constants
  W0 = 0x9E3779B9, W1 = 0xBB67AE85 (mod 2^32).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) integers < 2^32; key: (..., 2). Returns (..., 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    c = np.broadcast_to(c, np.broadcast_shapes(c.shape, k.shape[:-1] + (4,))).copy()
    k0 = np.broadcast_to(k[..., 0], c.shape[:-1]).copy()
    k1 = np.broadcast_to(k[..., 1], c.shape[:-1]).copy()
    x0, x1, x2, x3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * x0            # < 2^64, exact in uint64
        p1 = M1 * x2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def seed_key(seed: int):
    """64-bit seed -> Philox key words (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64)


def pick_index(word, deg):
    """Map a uniform 32-bit word to a neighbour position in [0, deg): floor(word*deg / 2^32)."""
    return (np.asarray(word, dtype=np.uint64) * np.asarray(deg, dtype=np.uint64)) >> S32
