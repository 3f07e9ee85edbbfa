"""FASTQ / FASTA text to (reads, offsets) — TEST INFRASTRUCTURE ONLY (the
oracle of the device parser; the product library never imports it).

Written line by line in plain Python, from the definitions of the two formats:
* FASTQ (Sanger): records of exactly four lines: '@' + name, the sequence,
  '+' (optionally the name again), the quality string. Multi-line FASTQ is not
  accepted.
* FASTA: a record is a '>' header line followed by any number of sequence
  lines (possibly none), which are concatenated.
Rules shared with the device parser: newline and carriage-return bytes at the
start and end of the text are ignored; carriage returns are dropped from
sequence lines (CRLF files); every other byte of a sequence line is kept as it
is (the counter decides which bytes are bases). Format 0 picks FASTQ when the
first kept byte is '@' and FASTA when it is '>'.
"""
from __future__ import annotations

import numpy as np

FASTQ, FASTA = 1, 2


class ParseError(ValueError):
    pass


def parse(text: bytes, fmt: int = 0):
    """Returns (reads uint8[n_bases], offsets uint64[n_records + 1], fmt)."""
    t = bytes(text).strip(b"\r\n")
    if not t:
        return np.zeros(0, np.uint8), np.zeros(1, np.uint64), fmt
    if fmt == 0:
        if t[:1] == b"@":
            fmt = FASTQ
        elif t[:1] == b">":
            fmt = FASTA
        else:
            raise ParseError("text starts with neither '@' nor '>'")
    lines = t.split(b"\n")
    seqs = []
    if fmt == FASTQ:
        if len(lines) % 4:
            raise ParseError("%d lines is not a whole number of 4-line records" % len(lines))
        for r in range(len(lines) // 4):
            if not lines[4 * r].startswith(b"@"):
                raise ParseError("line %d does not start with '@'" % (4 * r))
            if not lines[4 * r + 2].startswith(b"+"):
                raise ParseError("line %d does not start with '+'" % (4 * r + 2))
            seqs.append(lines[4 * r + 1].replace(b"\r", b""))
    elif fmt == FASTA:
        if not lines[0].startswith(b">"):
            raise ParseError("FASTA text does not start with '>'")
        for ln in lines:
            if ln.startswith(b">"):
                seqs.append([])
            else:
                seqs[-1].append(ln.replace(b"\r", b""))
        seqs = [b"".join(s) for s in seqs]
    else:
        raise ParseError("unknown format %d" % fmt)
    offsets = np.zeros(len(seqs) + 1, np.uint64)
    np.cumsum([len(s) for s in seqs], out=offsets[1:])
    reads = np.frombuffer(b"".join(seqs), dtype=np.uint8).copy()
    return reads, offsets, fmt
