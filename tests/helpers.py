"""Test-side helpers written directly from definitions (no shared code with oracle or GPU path)."""
from __future__ import annotations

import numpy as np

VALID = np.zeros(256, dtype=bool)
for _c in b"ACGTacgt":
    VALID[_c] = True


def to_arrays(reads: list[str]):
    data = "".join(reads).encode("latin-1")
    offs = np.zeros(len(reads) + 1, dtype=np.uint64)
    np.cumsum([len(r) for r in reads], out=offs[1:])
    return np.frombuffer(data, dtype=np.uint8).copy(), offs


def valid_windows_np(reads: np.ndarray, offsets: np.ndarray, k: int) -> int:
    """Windows whose k bytes are all bases, counted from runs of valid bytes per read."""
    total = 0
    base = int(offsets[0])
    v = VALID[reads]
    for a, b in zip(offsets[:-1].astype(np.int64), offsets[1:].astype(np.int64)):
        seg = v[a - base:b - base]
        if seg.size < k:
            continue
        # run lengths of True
        padded = np.concatenate([[False], seg, [False]])
        d = np.diff(padded.astype(np.int8))
        starts = np.flatnonzero(d == 1)
        ends = np.flatnonzero(d == -1)
        runs = ends - starts
        total += int(np.maximum(runs - k + 1, 0).sum())
    return total


def rc_int(key: int, k: int) -> int:
    """Reverse complement of an encoded k-mer, base by base."""
    out = 0
    for j in range(k):
        b = (key >> (2 * j)) & 3
        out = out * 4 + (3 - b)
    return out


def keys_as_ints(keys: np.ndarray, k: int) -> list[int]:
    """Keys as Python ints: one word each (k <= 32), or rows of words, least
    significant first."""
    if keys.ndim == 2:
        return [sum(int(w) << (64 * i) for i, w in enumerate(row)) for row in keys]
    return [int(x) for x in keys]


def ints_as_keys(ints: list[int], k: int) -> np.ndarray:
    """Inverse of keys_as_ints for the width k uses (1, 2 or 4 words)."""
    w = 1 if k <= 32 else (2 if k <= 64 else 4)
    rows = [[(x >> (64 * i)) & (2**64 - 1) for i in range(w)] for x in ints]
    arr = np.array(rows, dtype=np.uint64).reshape(len(ints), w)
    return arr[:, 0].copy() if w == 1 else arr


def revcomp_bytes(reads: np.ndarray, offsets: np.ndarray):
    """Reverse-complement every read (A<->T, C<->G, case kept, other bytes unchanged)."""
    table = np.arange(256, dtype=np.uint8)
    for a, b in [(b"A", b"T"), (b"C", b"G"), (b"a", b"t"), (b"c", b"g")]:
        table[a[0]] = b[0]
        table[b[0]] = a[0]
    out = np.empty_like(reads)
    base = int(offsets[0])
    for a, b in zip(offsets[:-1].astype(np.int64), offsets[1:].astype(np.int64)):
        out[a - base:b - base] = table[reads[a - base:b - base][::-1]]
    return out


def merge_sum(parts):
    """Sum several sorted (keys, counts) results into one (dict based; tiny/moderate sizes)."""
    acc = {}
    for keys, cnt in parts:
        kk = [tuple(x) for x in keys.tolist()] if keys.ndim == 2 else keys.tolist()
        for key, c in zip(kk, cnt.tolist()):
            acc[key] = acc.get(key, 0) + c
    items = sorted(acc.items(), key=lambda kv: kv[0][::-1] if isinstance(kv[0], tuple) else kv[0])
    return items


def de_bruijn(k: int, alphabet: str = "ACGT") -> str:
    """Linearised de Bruijn sequence B(|alphabet|, k) by the FKM (Lyndon word) construction."""
    n = len(alphabet)
    a = [0] * (n * k)
    seq: list[int] = []

    def db(t: int, p: int):
        if t > k:
            if k % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, n):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    s = "".join(alphabet[i] for i in seq)
    return s + s[:k - 1]
