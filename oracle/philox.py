"""Philox4x32-10 counter-based generator (test infrastructure: CPU oracle).

Written from the published definition in J. K. Salmon, M. A. Moraes,
R. O. Dror and D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11, Sec. 4.2 (the Philox S-box): a 4-word counter and a 2-word key;
each of the 10 rounds multiplies words 0 and 2 by the two round
multipliers, keeps the high and low halves of the 64-bit products, xors
the high halves with words 1 and 3 and with the round key, and permutes;
between rounds the key is advanced by the two Weyl constants.

The FAMST paper (Alg. 3) only says that endpoints are drawn at random from
each component; this generator fixes that draw so that two independent
implementations produce the same samples.
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9  # golden ratio
PHILOX_W1 = 0xBB67AE85  # sqrt(3) - 1


def philox4x32_10(ctr, key):
    """Return the 4 output words for counter ``ctr`` (4 ints) and ``key``
    (2 ints); every word is an unsigned 32-bit integer."""
    c0, c1, c2, c3 = (int(x) & MASK32 for x in ctr)
    k0, k1 = (int(x) & MASK32 for x in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return c0, c1, c2, c3


def seed_key(seed: int):
    """Split a 64-bit seed into the (low, high) key words."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def uniform_index(r: int, size: int) -> int:
    """Map a 32-bit word to {0..size-1} by multiply-shift: (r * size) >> 32."""
    return (int(r) * int(size)) >> 32
