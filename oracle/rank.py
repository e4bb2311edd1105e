"""Rank statistics and selection rules -- oracle side, test infrastructure only.

* Spearman's rank correlation: the Pearson correlation of the two rank
  vectors, tied values sharing the average of the ranks they span.
* Prescreen and survivor selection take the k best of a key vector, ties to
  the lower index.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10

TAG_PRESCREEN = 10
TAG_AUDIT = 9


def average_ranks(x) -> np.ndarray:
    """Ranks 1..n, ties get the mean of the positions they occupy."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    order = sorted(range(n), key=lambda i: (x[i], i))
    ranks = np.empty(n)
    i = 0
    while i < n:
        j = i
        while j + 1 < n and x[order[j + 1]] == x[order[i]]:
            j += 1
        r = (i + j) / 2.0 + 1.0
        for q in range(i, j + 1):
            ranks[order[q]] = r
        i = j + 1
    return ranks


def spearman(a, b) -> float:
    ra, rb = average_ranks(a), average_ranks(b)
    ra = ra - ra.mean()
    rb = rb - rb.mean()
    den = np.sqrt((ra * ra).sum() * (rb * rb).sum())
    return float((ra * rb).sum() / den) if den > 0 else 0.0


def smallest_k(keys, k: int) -> list:
    """Indices of the k smallest keys, ties to the lower index, in that order."""
    keys = np.asarray(keys, dtype=np.float64)
    return sorted(range(keys.size), key=lambda i: (keys[i], i))[:k]


def random_keys(n: int, g: int, tag: int, seed: int) -> np.ndarray:
    """One uniform u32 word per offspring (block (i, 0, g, tag) word 0)."""
    i = np.arange(n, dtype=np.uint64)
    w0, _, _, _ = philox4x32_10(i, 0, g, tag, seed)
    return w0.astype(np.float64)
