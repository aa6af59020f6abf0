"""Philox4x32-10 counter-based generator -- test infrastructure.

Written from the definition in Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter is mixed by
ten rounds of a multiply-based bijection keyed by a 2x32-bit key, with a
Weyl-sequence bump of the key between rounds.

One round on counter (c0, c1, c2, c3) with key (k0, k1):
    (hi0, lo0) = 64-bit product M0 * c0 split into halves
    (hi1, lo1) = M1 * c2
    result     = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
Multipliers M0 = 0xD2511F53, M1 = 0xCD9E8D57; key bumps W0 = 0x9E3779B9,
W1 = 0xBB67AE85 (added mod 2^32 after each round but the last).

Fixed mappings from the 32-bit outputs used by the generation step:
  integer in [0, n):  (u * n) >> 32            (multiply-high, bias < n / 2^32)
  unit float [0, 1):  (u >> 8) * 2^-24         (exact in binary32 and binary64)
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Scalar form: ctr = 4 ints, key = 2 ints -> tuple of 4 uint32 ints."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised form over numpy arrays of counters (uint32 semantics)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK)
    k1 = np.uint64(int(k1) & MASK)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    mask = np.uint64(MASK)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def below(u: int, n: int) -> int:
    """Integer in [0, n) from one 32-bit output."""
    return (int(u) * int(n)) >> 32


def unit(u: int) -> float:
    """Unit float in [0, 1) with 24 random bits."""
    return float(int(u) >> 8) * (2.0 ** -24)


class Stream:
    """Draws of one individual: draw j is word j % 4 of the block j // 4.

    The block counter is (index, generation, block, tag); the key is the
    64-bit seed split into two 32-bit halves (low word first).
    """

    def __init__(self, seed: int, index: int, generation: int, tag: int):
        self.key = (seed & MASK, (seed >> 32) & MASK)
        self.index = index & MASK
        self.gen = generation & MASK
        self.tag = tag & MASK
        self._blk = -1
        self._words = None

    def draw(self, j: int) -> int:
        b = j // 4
        if b != self._blk:
            self._words = philox4x32_10((self.index, self.gen, b, self.tag), self.key)
            self._blk = b
        return self._words[j % 4]
