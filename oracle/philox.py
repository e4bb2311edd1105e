"""Philox4x32-10 counter-based generator -- oracle side, test infrastructure only.

Written from Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers: As Easy
as 1, 2, 3" (SC'11): a 4 x 32-bit counter is mixed by ten rounds, each of
which multiplies words 0 and 2 by the published multipliers, swaps the
products' high and low halves across the counter and xors in the key; the
two-word key is advanced by the published Weyl increments between rounds.

The GA uses counters (a, b, generation, stream tag) and the key (seed low
32 bits, seed high 32 bits); see ``oracle.ga`` for how each operator draws.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_MUL0 = np.uint64(0xD2511F53)
_MUL1 = np.uint64(0xCD9E8D57)
_WEYL0 = np.uint64(0x9E3779B9)
_WEYL1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, seed: int):
    """Vectorised Philox4x32-10. Counters broadcast; returns 4 uint32 arrays."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64(seed >> 32)
    x = [np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3)]
    x = np.broadcast_arrays(*x)
    x = [np.array(v, dtype=np.uint64) for v in x]
    for r in range(10):
        if r:
            k0 = (k0 + _WEYL0) & _MASK
            k1 = (k1 + _WEYL1) & _MASK
        p0 = _MUL0 * x[0]          # < 2^64, exact in uint64
        p1 = _MUL1 * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return tuple(v.astype(np.uint32) for v in x)


def philox_block(ctr, seed: int):
    """One counter (tuple of 4 ints) -> list of 4 Python ints."""
    out = philox4x32_10(*[np.uint64(c) for c in ctr], seed=seed)
    return [int(v) for v in out]
