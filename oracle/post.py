"""Uses of a k-mer histogram, written from their definitions — TEST
INFRASTRUCTURE ONLY (tests import it; the product path never does).

A histogram here is (keys, counts) as ``oracle.count`` returns it: keys
uint64[D] (one word) or uint64[D, w] (w words, least significant first),
sorted ascending, unique, with uint32 counts.

* spectrum: how many keys have each count (the k-mer spectrum that downstream
  uses of the histogram read, Section I), the last bin taking every count
  at or above it;
* filter_min_count: the pairs whose count is at least a minimum, in order;
* merge: the histogram of the union of two read collections from their two
  histograms (a histogram is additive over any split of the reads).
"""
from __future__ import annotations

import numpy as np


def _rows(keys: np.ndarray) -> list:
    """Keys as Python ints (words least significant first)."""
    if keys.ndim == 1:
        return [int(x) for x in keys]
    return [sum(int(w) << (64 * i) for i, w in enumerate(row)) for row in keys]


def _words(ints: list, w: int) -> np.ndarray:
    arr = np.array([[(x >> (64 * i)) & (2**64 - 1) for i in range(w)] for x in ints],
                   dtype=np.uint64).reshape(len(ints), w)
    return arr[:, 0].copy() if w == 1 else arr


def spectrum(counts: np.ndarray, max_count: int) -> np.ndarray:
    """hist[c] = number of keys with count c for 1 <= c < max_count;
    hist[max_count] = number with count >= max_count; hist[0] = 0."""
    hist = np.zeros(max_count + 1, dtype=np.uint64)
    for c in counts.tolist():
        hist[min(int(c), max_count)] += 1
    return hist


def filter_min_count(keys: np.ndarray, counts: np.ndarray, min_count: int):
    """The pairs with count >= min_count, in their order."""
    keep = [i for i, c in enumerate(counts.tolist()) if c >= min_count]
    return keys[keep], counts[keep]


def merge(a_keys: np.ndarray, a_counts: np.ndarray, b_keys: np.ndarray, b_counts: np.ndarray,
          words: int):
    """Union of the keys of two histograms, counts added where a key is in
    both, in ascending key order. Raises OverflowError past 2^32 - 1."""
    acc: dict = {}
    for ks, cs in ((a_keys, a_counts), (b_keys, b_counts)):
        for key, c in zip(_rows(ks), cs.tolist()):
            acc[key] = acc.get(key, 0) + int(c)
    order = sorted(acc)
    tot = [acc[x] for x in order]
    if tot and max(tot) > 0xFFFFFFFF:
        raise OverflowError("a merged count exceeds 2^32 - 1")
    return _words(order, words), np.array(tot, dtype=np.uint32)
