"""Pins of the result-use oracles (oracle/post.py: spectrum, minimum-count
filter, merge) against closed forms, string brute force and the additivity
of the histogram over a split of the reads. No GPU."""
from collections import Counter

import numpy as np
import pytest

import oracle
import synth
from oracle import brute, post
from helpers import de_bruijn, to_arrays


def test_spectrum_closed_forms():
    # de Bruijn B(4, k), odd k: every canonical class is seen exactly twice
    k = 5
    r, o = to_arrays([de_bruijn(k)])
    keys, cnt = oracle.count(r, o, k)
    h = post.spectrum(cnt, 10)
    assert h[2] == 4 ** k // 2 and h.sum() == 4 ** k // 2 and h[0] == 0
    # even k: palindromes once, the others twice
    k = 4
    r, o = to_arrays([de_bruijn(k)])
    keys, cnt = oracle.count(r, o, k)
    h = post.spectrum(cnt, 10)
    assert h[1] == 4 ** (k // 2) and h[2] == (4 ** k - 4 ** (k // 2)) // 2
    # homopolymer of length L: one key of count L - k + 1, in the last bin when it is large
    r, o = to_arrays(["A" * 200])
    keys, cnt = oracle.count(r, o, 31)
    assert list(post.spectrum(cnt, 1000)[[0, 170]]) == [0, 1]
    assert post.spectrum(cnt, 100)[100] == 1 and post.spectrum(cnt, 100).sum() == 1


def test_spectrum_sums_against_brute_force():
    text, offs = synth.ragged_reads(5, 200, 0, 80, b"ACGTACGTNacgt")
    k = 7
    want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
    keys, cnt = oracle.count(text, offs, k)
    tally = Counter(c for _, c in want)
    h = post.spectrum(cnt, 4)
    assert h[1] == tally[1] and h[2] == tally[2] and h[3] == tally[3]
    assert h[4] == sum(v for c, v in tally.items() if c >= 4)
    big = post.spectrum(cnt, 10_000)
    assert int(big.sum()) == len(want)
    assert int(sum(c * int(v) for c, v in enumerate(big))) == sum(c for _, c in want)


@pytest.mark.parametrize("k", [11, 40, 90])
def test_filter_against_brute_force(k):
    text, offs = synth.ragged_reads(7 + k, 150, k, 3 * k, b"AACGTTN")
    want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
    keys, cnt = oracle.count(text, offs, k)
    for m in (1, 2, 3, 50):
        fk, fc = post.filter_min_count(keys, cnt, m)
        exp = [(x, c) for x, c in want if c >= m]
        from helpers import keys_as_ints
        assert list(zip(keys_as_ints(fk, k), fc.tolist())) == exp


@pytest.mark.parametrize("k", [21, 31, 55, 64, 99])
def test_merge_is_the_count_of_the_union(k):
    """count(R1 + R2) == merge(count(R1), count(R2)), the halves split at every
    position class (first read, middle, last read)."""
    text, offs = synth.ragged_reads(31 + k, 120, 0, 2 * k + 40, b"ACGTACGTACGTN")
    whole = oracle.count(text, offs, k)
    n = offs.size - 1
    for cut in (0, 1, n // 2, n):
        a = oracle.count(text[:int(offs[cut])], offs[:cut + 1], k)
        bo = offs[cut:] - offs[cut]
        b = oracle.count(text[int(offs[cut]):], bo, k)
        mk, mc = post.merge(a[0], a[1], b[0], b[1], oracle.key_words(k))
        assert np.array_equal(mk, whole[0]) and np.array_equal(mc, whole[1])


def test_merge_overflow_is_reported():
    a = (np.array([5], dtype=np.uint64), np.array([0xFFFFFFFF], dtype=np.uint32))
    b = (np.array([5], dtype=np.uint64), np.array([1], dtype=np.uint32))
    with pytest.raises(OverflowError):
        post.merge(a[0], a[1], b[0], b[1], 1)
    mk, mc = post.merge(a[0], a[1], np.array([6], np.uint64), np.array([1], np.uint32), 1)
    assert mk.tolist() == [5, 6] and mc.tolist() == [0xFFFFFFFF, 1]
