"""Philox4x32-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key; each of the 10 rounds
multiplies words 0 and 2 by two fixed 32-bit multipliers, forms the next
counter from the high halves xor'ed with the other words and the round key and
the low halves, and the key is bumped by two Weyl constants between rounds.

Use in the trajectory ensemble: one draw per (trajectory k, noise site s),
    key = (seed mod 2^32, seed >> 32),   counter = (k mod 2^32, k >> 32, s, 0),
    r   = word 0 of the output.
The draw depends only on (seed, k, s): never on how trajectories are batched.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ctr: (..., 4) integer array of 32-bit words; key: (..., 2).
    Returns a (..., 4) uint64 array of 32-bit output words."""
    c = np.asarray(ctr, dtype=np.uint64) & np.uint64(MASK)
    k = np.asarray(key, dtype=np.uint64) & np.uint64(MASK)
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    m = np.uint64(MASK)
    for rnd in range(10):
        p0 = np.uint64(M0) * c0          # < 2^64, exact in uint64
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & m, lo1, (hi0 ^ c3 ^ k1) & m, lo0
        if rnd < 9:
            k0 = (k0 + np.uint64(W0)) & m
            k1 = (k1 + np.uint64(W1)) & m
    return np.stack([c0, c1, c2, c3], axis=-1)


def site_draws(seed, k0, K, S):
    """uint64 array [K, S] of 32-bit draws r(k, s) for k = k0..k0+K-1."""
    k = np.arange(k0, k0 + K, dtype=np.uint64)[:, None]
    s = np.arange(S, dtype=np.uint64)[None, :]
    ctr = np.stack(np.broadcast_arrays(k & np.uint64(MASK), k >> np.uint64(32), s,
                                       np.zeros_like(s)), axis=-1)
    key = np.array([seed & MASK, (seed >> 32) & MASK], dtype=np.uint64)
    key = np.broadcast_to(key, ctr.shape[:-1] + (2,))
    return philox4x32_10(ctr, key)[..., 0]
