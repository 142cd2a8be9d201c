"""Philox4x32-10 counter-based generator, float64 oracle side (test-only).

Definition followed: Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11, Sec. 3 (Philox-4x32 S-box, round key schedule,
10 rounds).  One round maps the counter (c0, c1, c2, c3) under key (k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with M0 = 0xD2511F53, M1 = 0xCD9E8D57; between rounds the key is bumped by the
Weyl constants (0x9E3779B9, 0xBB67AE85) modulo 2**32.

This module is vectorised over numpy arrays of counters; it shares no code
with the device implementation.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
ROUNDS = 10


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Apply Philox4x32-`rounds` to counters (c0..c3) under key (k0, k1).

    All arguments are broadcastable integer arrays (or ints) with values in
    [0, 2**32).  Returns a tuple of four uint32 arrays (the output block).
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = (np.array(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(rounds):
        p0 = M0 * c0            # < 2**64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        if r + 1 < rounds:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))
