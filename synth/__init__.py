"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's synthetic data sets (Table V: reads of 150 bp sampled from a
uniform random genome of 2^XY bases) are produced there by an Illumina read
simulator; here a small C++ generator (``kcsynth.cpp``) stands in for it with
substitution-only errors, optional 'N' bases and optional repeat families.

This module is input synthesis only. It holds no k-mer arithmetic and is the
one place both the CPU oracle tests and the GPU path take their inputs from.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kcsynth.cpp")
_SO = os.path.join(_HERE, "libkcsynth.so")
_lock = threading.Lock()
_lib = None

CONFIG_SEED_BASE = 0x6B6D657200000000  # "kmer" in the high word, config index in the low word


def build(force: bool = False) -> str:
    """Compile the generator into ``synth/libkcsynth.so`` with g++."""
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
            u64, p = ctypes.c_uint64, ctypes.c_void_p
            L.kcsynth_genome_length.restype = u64
            L.kcsynth_genome_length.argtypes = [u64, ctypes.c_uint32, p, p]
            L.kcsynth_genome.restype = None
            L.kcsynth_genome.argtypes = [u64, u64, ctypes.c_uint32, p, p, p, p]
            L.kcsynth_reads.restype = None
            L.kcsynth_reads.argtypes = [u64, u64, p, u64, u64, u64, p, p,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, p]
            L.kcsynth_random_text.restype = None
            L.kcsynth_random_text.argtypes = [u64, u64, ctypes.c_char_p, ctypes.c_int, u64, p]
            _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def genome(seed: int, backbone_len: int, families=()) -> np.ndarray:
    """Uniform ACGT backbone plus inserted diverged repeat copies.

    ``families`` is a sequence of (length, copies, divergence).
    Returns an ASCII uint8 array.
    """
    L = lib()
    nf = len(families)
    flen = np.array([f[0] for f in families] or [0], dtype=np.uint64)
    fcop = np.array([f[1] for f in families] or [0], dtype=np.uint64)
    fdiv = np.array([f[2] for f in families] or [0.0], dtype=np.float64)
    G = L.kcsynth_genome_length(backbone_len, nf, _ptr(flen), _ptr(fcop))
    out = np.empty(G, dtype=np.uint8)
    L.kcsynth_genome(seed, backbone_len, nf, _ptr(flen), _ptr(fcop), _ptr(fdiv), _ptr(out))
    return out


def reads(genome_arr: np.ndarray, n_reads: int, read_len: int = 150, lens=None,
          err_rate: float = 0.0, n_rate: float = 0.0, seed: int = 1, stream_base: int = 0,
          threads: int | None = None):
    """Sample reads from a genome. Returns (reads uint8[total], offsets uint64[n+1])."""
    L = lib()
    if lens is not None:
        lens = np.ascontiguousarray(lens, dtype=np.uint64)
        assert lens.shape[0] == n_reads
        offsets = np.zeros(n_reads + 1, dtype=np.uint64)
        np.cumsum(lens, out=offsets[1:])
    else:
        offsets = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(read_len)
    out = np.empty(int(offsets[-1]), dtype=np.uint8)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if n_reads:
        L.kcsynth_reads(seed, stream_base, _ptr(genome_arr), genome_arr.shape[0], n_reads,
                        read_len, _ptr(lens), _ptr(offsets), err_rate, n_rate, threads, _ptr(out))
    return out, offsets


def random_text(seed: int, n: int, alphabet: bytes = b"ACGT", stream: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    if n:
        lib().kcsynth_random_text(seed, stream, alphabet, len(alphabet), n, _ptr(out))
    return out


def ragged_reads(seed: int, n_reads: int, min_len: int, max_len: int,
                 alphabet: bytes = b"ACGT") -> tuple[np.ndarray, np.ndarray]:
    """Reads of i.i.d. bytes with uniform random lengths in [min_len, max_len]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.integers(min_len, max_len + 1, size=n_reads, dtype=np.int64).astype(np.uint64)
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    text = random_text(seed, int(offsets[-1]), alphabet, stream=7)
    return text, offsets


from .configs import (CONFIGS, c4_sample, c4_set_reads, c4_sets, c5_job_reads,  # noqa: E402,F401
                      c5_jobs, c5_sample, family_layout, make_config, waves)


def to_fastq(reads_arr: np.ndarray, offsets: np.ndarray, seed: int = 1, crlf: bool = False,
             plus_name: bool = False, trailing: bytes = b"\n") -> bytes:
    """FASTQ text of the given reads: four lines per record (@name, sequence,
    +[name], quality). Qualities are random Phred+33 characters '!'..'J', so
    they include 'A', 'C' and 'G' and a parser must tell the lines apart by
    position, not content."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nl = b"\r\n" if crlf else b"\n"
    offs = np.asarray(offsets, dtype=np.uint64)
    n = offs.size - 1
    qual = rng.integers(33, 75, size=int(offs[-1] - offs[0]), dtype=np.uint8).tobytes()
    data = np.asarray(reads_arr, dtype=np.uint8).tobytes()
    b0 = int(offs[0])
    parts = []
    for i in range(n):
        s, e = int(offs[i]), int(offs[i + 1])
        name = b"r%d len=%d" % (i, e - s)
        parts += [b"@", name, nl, data[s:e], nl, b"+", name if plus_name else b"", nl,
                  qual[s - b0:e - b0], nl]
    text = b"".join(parts)
    return text[:-len(nl)] + trailing if n else trailing


def to_fasta(reads_arr: np.ndarray, offsets: np.ndarray, width: int = 60, crlf: bool = False,
             trailing: bytes = b"\n") -> bytes:
    """FASTA text of the given reads: a '>' header line per record, the sequence
    wrapped at ``width`` bases per line (width 0: one line)."""
    nl = b"\r\n" if crlf else b"\n"
    offs = np.asarray(offsets, dtype=np.uint64)
    n = offs.size - 1
    data = np.asarray(reads_arr, dtype=np.uint8).tobytes()
    parts = []
    for i in range(n):
        s, e = int(offs[i]), int(offs[i + 1])
        parts += [b">seq%d some description" % i, nl]
        w = width if width > 0 else max(1, e - s)
        for p in range(s, e, w):
            parts += [data[p:min(e, p + w)], nl]
    text = b"".join(parts)
    return text[:-len(nl)] + trailing if n else trailing
