"""Pins of the FASTQ / FASTA parsing oracle: hand-written texts with their
sequences written out by hand (tests/golden/fastx_examples.json), malformed
texts that must be refused, and the round trip reads -> text -> reads through
the synthetic formatters (whose output the oracle has to undo exactly)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import fastx

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "fastx_examples.json")))


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=lambda c: c["name"])
def test_golden(case):
    reads, offs, fmt = fastx.parse(case["text"].encode(), case["format"])
    seqs = [reads[int(offs[i]):int(offs[i + 1])].tobytes().decode()
            for i in range(offs.size - 1)]
    assert seqs == case["expect"]
    assert int(offs[0]) == 0
    if case["expect"]:
        assert fmt == case["format_out"]


@pytest.mark.parametrize("case", GOLDEN["errors"], ids=lambda c: c["name"])
def test_golden_errors(case):
    with pytest.raises(fastx.ParseError):
        fastx.parse(case["text"].encode(), case["format"])


@pytest.mark.parametrize("crlf", [False, True])
@pytest.mark.parametrize("trailing", [b"", b"\n", b"\r\n\n"])
def test_round_trip(crlf, trailing):
    reads, offs = synth.ragged_reads(11, 300, 0, 90, alphabet=b"ACGTNacgtRY")
    texts = [synth.to_fastq(reads, offs, seed=2, crlf=crlf, trailing=trailing),
             synth.to_fastq(reads, offs, seed=3, crlf=crlf, plus_name=True, trailing=trailing),
             synth.to_fasta(reads, offs, width=60, crlf=crlf, trailing=trailing),
             synth.to_fasta(reads, offs, width=1, crlf=crlf, trailing=trailing),
             synth.to_fasta(reads, offs, width=0, crlf=crlf, trailing=trailing)]
    for i, t in enumerate(texts):
        r, o, f = fastx.parse(t)
        assert f == (fastx.FASTQ if i < 2 else fastx.FASTA)
        assert np.array_equal(r, reads) and np.array_equal(o, offs), i


def test_fastq_qualities_hold_base_letters():
    """The formatter's qualities include 'A', 'C', 'G': a parser that kept
    quality lines would change the reads."""
    reads, offs = synth.ragged_reads(5, 200, 50, 60)
    t = synth.to_fastq(reads, offs, seed=9)
    quals = t.split(b"\n")[3::4]
    assert any(c in q for q in quals for c in b"ACG")
