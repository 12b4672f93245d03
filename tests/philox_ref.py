"""Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from its published definition for the tests: a
counter-based generator, so a random value is a pure function of (counter,
key).  Ten rounds; each round multiplies words 0 and 2 of the counter by the
constants 0xD2511F53 and 0xCD9E8D57, takes high and low halves of the 64-bit
products, and mixes in the key, which is bumped between rounds by the Weyl
constants 0x9E3779B9 and 0xBB67AE85.  Vectorized over counters with numpy."""

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32 counters; key: (2,) uint32.  Returns (..., 4) uint32."""
    c = [np.asarray(ctr[..., j], dtype=np.uint32).astype(np.uint64) for j in range(4)]
    k0, k1 = np.uint32(key[0]), np.uint32(key[1])
    for r in range(10):
        if r:
            k0 = np.uint32((int(k0) + int(W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(W1)) & 0xFFFFFFFF)
        p0 = c[0] * M0
        p1 = c[2] * M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return np.stack([v.astype(np.uint32) for v in c], axis=-1)
