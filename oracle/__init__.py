"""CPU oracle for canonical k-mer counting — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never imports,
links or calls it.

What is here, each written from the definition of the k-mer histogram
(Section II; Algorithm 1 counts it serially by sorting):

* ``liboracle.so`` (``kc_oracle.cpp``): every valid window's forward and
  reverse-complement values decoded from its own bytes, the smaller kept,
  keys sorted and tallied; a std::map tally as a cross-check; a tally of
  chosen keys and a tally restricted to a range of top key bits, for inputs
  too large to tally at once.
* ``post.py``: the uses of a result (spectrum, minimum-count filter, merge of
  two results) as plain numpy / dict code.
* ``brute.py``: pure-Python string brute force for tiny inputs.
* ``fastx.py``: FASTQ / FASTA parsing by the formats' definitions.

None shares code with the GPU path. Parity pins: tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.cpp")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_SO)
            p, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
            L.oracle_valid_windows.restype = u64
            L.oracle_valid_windows.argtypes = [p, p, u64, i32]
            L.oracle_count_sort.restype = i32
            L.oracle_count_sort.argtypes = [p, p, u64, i32, i32, p, p, u64, p]
            L.oracle_count_map.restype = i32
            L.oracle_count_map.argtypes = [p, p, u64, i32, p, p, u64, p]
            L.oracle_count_range.restype = i32
            L.oracle_count_range.argtypes = [p, p, u64, i32, i32, i32, u64, u64, p, p, u64, p]
            L.oracle_count_selected.restype = i32
            L.oracle_count_selected.argtypes = [p, p, u64, i32, i32, p, u64, p]
            _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _prep(reads, offsets):
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if reads.size == 0:
        reads = np.zeros(1, dtype=np.uint8)
    return reads, offsets


def max_windows(offsets, k: int) -> int:
    """Number of length-k windows (valid or not): sum over reads of max(0, len-k+1)."""
    lens = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(np.maximum(lens - k + 1, 0).sum())


def valid_windows(reads, offsets, k: int) -> int:
    reads, offsets = _prep(reads, offsets)
    return int(lib().oracle_valid_windows(_p(reads), _p(offsets), offsets.size - 1, k))


def key_words(k: int) -> int:
    """64-bit words per key: 1 (k <= 32), 2 (k <= 64), 4 (k <= 128)."""
    return 1 if k <= 32 else (2 if k <= 64 else 4)


def count(reads, offsets, k: int, threads: int | None = None, method: str = "sort"):
    """Sorted canonical (k-mer, count) pairs.

    Returns (keys, counts): keys uint64[D] for k <= 32, uint64[D, w] with the
    w = 2 (k <= 64) or 4 (k <= 128) words of a key least significant first;
    counts uint32[D].
    """
    reads, offsets = _prep(reads, offsets)
    n = offsets.size - 1
    words = key_words(k) if 1 <= k <= 128 else 1
    cap = max(1, max_windows(offsets, k))
    keys = np.empty(cap * words, dtype=np.uint64)
    cnt = np.empty(cap, dtype=np.uint32)
    n_out = np.zeros(1, dtype=np.uint64)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if method == "sort":
        rc = lib().oracle_count_sort(_p(reads), _p(offsets), n, k, threads, _p(keys), _p(cnt),
                                     cap, _p(n_out))
    elif method == "map":
        rc = lib().oracle_count_map(_p(reads), _p(offsets), n, k, _p(keys), _p(cnt), cap,
                                    _p(n_out))
    else:
        raise ValueError(method)
    if rc != 0:
        raise RuntimeError("oracle error %d" % rc)
    d = int(n_out[0])
    keys = keys[:d * words].copy()
    return (keys.reshape(d, words) if words > 1 else keys), cnt[:d].copy()


def count_range(reads, offsets, k: int, bits: int, lo: int, hi: int,
                threads: int | None = None, capacity: int | None = None):
    """The histogram restricted to keys whose top `bits` bits (of the 2k-bit
    key) lie in [lo, hi); same layout as count(). capacity bounds the pairs
    of the slice (default: every window)."""
    reads, offsets = _prep(reads, offsets)
    n = offsets.size - 1
    words = key_words(k)
    cap = max(1, capacity if capacity is not None else max_windows(offsets, k))
    keys = np.empty(cap * words, dtype=np.uint64)
    cnt = np.empty(cap, dtype=np.uint32)
    n_out = np.zeros(1, dtype=np.uint64)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rc = lib().oracle_count_range(_p(reads), _p(offsets), n, k, threads, bits, lo, hi, _p(keys),
                                  _p(cnt), cap, _p(n_out))
    if rc != 0:
        raise RuntimeError("oracle error %d (n_out %d)" % (rc, int(n_out[0])))
    d = int(n_out[0])
    keys = keys[:d * words].copy()
    return (keys.reshape(d, words) if words > 1 else keys), cnt[:d].copy()


def count_selected(reads, offsets, k: int, keys, threads: int | None = None):
    """Count only the given canonical keys (uint64[m] or uint64[m, w] as count()
    returns them). Returns uint64[m]."""
    reads, offsets = _prep(reads, offsets)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    m = keys.shape[0]
    assert keys.size == m * key_words(k), "keys must hold %d word(s) each" % key_words(k)
    out = np.zeros(m, dtype=np.uint64)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rc = lib().oracle_count_selected(_p(reads), _p(offsets), offsets.size - 1, k, threads,
                                     _p(keys) if m else None, m, _p(out))
    if rc != 0:
        raise RuntimeError("oracle error %d" % rc)
    return out
