"""String brute force for tiny inputs — TEST INFRASTRUCTURE ONLY.

The k-mer histogram of Section II computed directly from its definition on
Python strings: every length-k substring made only of A/C/G/T (either case) is
upper-cased, replaced by the lexicographically smaller of itself and its
reverse complement, and tallied. The tally is then encoded with A=0, C=1,
G=2, T=3, first base most significant, and sorted. No bit arithmetic on
k-mers happens before the final encoding, so this shares no step with the
integer oracle or the GPU path.
"""
from __future__ import annotations

from collections import Counter

_COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
_CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def revcomp(s: str) -> str:
    return "".join(_COMP[c] for c in reversed(s))


def encode(s: str) -> int:
    v = 0
    for c in s:
        v = v * 4 + _CODE[c]
    return v


def count_strings(reads: list[str], k: int) -> list[tuple[int, int]]:
    tally: Counter = Counter()
    for r in reads:
        u = r.upper()
        for p in range(len(u) - k + 1):
            w = u[p:p + k]
            if all(c in _COMP for c in w):
                rc = revcomp(w)
                tally[min(w, rc)] += 1
    return sorted((encode(w), c) for w, c in tally.items())


def split_reads(reads_bytes: bytes, offsets) -> list[str]:
    offs = [int(x) for x in offsets]
    base = offs[0]
    return [reads_bytes[a - base:b - base].decode("latin-1") for a, b in zip(offs[:-1], offs[1:])]
