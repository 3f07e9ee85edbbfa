"""Pins of the CPU oracle against facts that do not come from the oracle itself.

The oracle follows Algorithm 1 ("Serial Algorithm") plus the canonical form;
these tests check it against hand-worked examples, a string brute force,
the de Bruijn closed form, homopolymers and invariants of the k-mer histogram
(Section II). None of them needs a GPU.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from helpers import (de_bruijn, ints_as_keys, keys_as_ints, merge_sum, rc_int, revcomp_bytes,
                     to_arrays, valid_windows_np)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
KS = [1, 2, 3, 4, 5, 8, 15, 16, 17, 21, 31, 32, 33, 55, 63, 64, 65, 77, 96, 97, 127, 128]


def _pairs(keys, cnt, k):
    return list(zip(keys_as_ints(keys, k), [int(c) for c in cnt]))


@pytest.mark.parametrize("method", ["sort", "map"])
def test_hand_examples(method):
    ex = json.load(open(GOLDEN))["examples"]
    for e in ex:
        r, o = to_arrays(e["reads"])
        keys, cnt = oracle.count(r, o, e["k"], method=method)
        got = _pairs(keys, cnt, e["k"])
        want_strings = [(brute.encode(s), c) for s, c in e["expect"]]
        assert got == want_strings, e["name"]
        assert [g[0] for g in got] == e["keys"], e["name"]


@pytest.mark.parametrize("k", KS)
def test_brute_force_random(k):
    # ragged reads with N, lowercase and an IUPAC code; some empty or shorter than k
    for seed in range(3):
        text, offs = synth.ragged_reads(1000 * k + seed, 40, 0, 3 * k + 20, b"ACGTACGTACGTacgtNR")
        want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
        for method in ("sort", "map"):
            keys, cnt = oracle.count(text, offs, k, threads=3, method=method)
            assert _pairs(keys, cnt, k) == want


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_de_bruijn_closed_form(k):
    s = de_bruijn(k)
    assert len(s) == 4 ** k + k - 1
    r, o = to_arrays([s])
    keys, cnt = oracle.count(r, o, k)
    pal = [key for key in keys_as_ints(keys, k) if rc_int(key, k) == key]
    expect_d = (4 ** k + 4 ** (k // 2)) // 2 if k % 2 == 0 else 4 ** k // 2
    assert len(keys) == expect_d
    assert int(cnt.sum()) == 4 ** k
    assert len(pal) == (4 ** (k // 2) if k % 2 == 0 else 0)
    for key, c in zip(keys_as_ints(keys, k), cnt.tolist()):
        assert c == (1 if rc_int(key, k) == key else 2)


@pytest.mark.parametrize("k", [1, 5, 31, 32, 33, 64, 65, 100, 128])
def test_homopolymers(k):
    L = 300
    for base, enc in [("A", 0), ("T", 0), ("C", brute.encode("C" * k)), ("G", brute.encode("C" * k))]:
        r, o = to_arrays([base * L])
        keys, cnt = oracle.count(r, o, k)
        assert keys_as_ints(keys, k) == [enc]
        assert cnt.tolist() == [L - k + 1]


@pytest.mark.parametrize("k", [3, 21, 31, 32, 33, 55, 65, 99, 128])
def test_invariants_on_synthetic_reads(k):
    g = synth.genome(11, 3000, [(200, 5, 0.02)])
    r, o = synth.reads(g, 300, 150, err_rate=0.01, n_rate=0.002, seed=5)
    keys, cnt = oracle.count(r, o, k)
    ints = keys_as_ints(keys, k)
    assert int(cnt.sum()) == valid_windows_np(r, o, k)
    assert int(cnt.sum()) == oracle.valid_windows(r, o, k)
    assert all(a < b for a, b in zip(ints, ints[1:]))
    assert all(x < 4 ** k and x <= rc_int(x, k) for x in ints)
    assert (cnt >= 1).all()
    # strand flip
    keys2, cnt2 = oracle.count(revcomp_bytes(r, o), o, k)
    assert np.array_equal(keys, keys2) and np.array_equal(cnt, cnt2)
    # read permutation
    perm = np.random.Generator(np.random.PCG64(3)).permutation(o.size - 1)
    lens = np.diff(o.astype(np.int64))[perm]
    chunks = [r[int(o[i]):int(o[i + 1])] for i in perm]
    r3 = np.concatenate(chunks)
    o3 = np.zeros_like(o)
    np.cumsum(lens, out=o3[1:])
    keys3, cnt3 = oracle.count(r3, o3, k)
    assert np.array_equal(keys, keys3) and np.array_equal(cnt, cnt3)
    # split additivity
    h = (o.size - 1) // 3
    a = oracle.count(r[:int(o[h])], o[:h + 1], k)
    oo = o[h:] - o[h]
    b = oracle.count(r[int(o[h]):], oo, k)
    merged = merge_sum([a, b])
    assert [m[1] for m in merged] == cnt.tolist()


def test_thread_count_and_nonzero_offset_base():
    g = synth.genome(12, 20000)
    r, o = synth.reads(g, 2000, 150, err_rate=0.005, seed=9)
    k1, c1 = oracle.count(r, o, 31, threads=1)
    k8, c8 = oracle.count(r, o, 31, threads=8)
    assert np.array_equal(k1, k8) and np.array_equal(c1, c8)
    # offsets that start past the beginning of the byte buffer
    o2 = o + np.uint64(1000)
    k2, c2 = oracle.count(r, o2, 31, threads=4)
    assert np.array_equal(k1, k2) and np.array_equal(c1, c2)


def test_selected_counts_match_full():
    g = synth.genome(13, 5000, [(300, 8, 0.01)])
    r, o = synth.reads(g, 500, 150, err_rate=0.01, n_rate=0.001, seed=2)
    for k in (21, 55, 100):
        keys, cnt = oracle.count(r, o, k)
        sel = np.arange(0, len(cnt), 7)
        got = oracle.count_selected(r, o, k, keys[sel])
        assert np.array_equal(got, cnt[sel].astype(np.uint64))
        # keys that cannot occur (not canonical: bigger than their revcomp) count 0
        absent = [x for x in (4 ** k - 1, 4 ** k - 2) if rc_int(x, k) < x]
        assert oracle.count_selected(r, o, k, ints_as_keys(absent, k)).tolist() == [0] * len(absent)


def test_bad_arguments():
    r, o = to_arrays(["ACGT"])
    for k in (0, 129):
        with pytest.raises(RuntimeError):
            oracle.count(r, o, k)
    with pytest.raises(RuntimeError):
        oracle.count(r, np.array([0, 3, 2], dtype=np.uint64), 2)


def test_generator_is_deterministic_and_thread_invariant():
    g1 = synth.genome(77, 10000, [(500, 3, 0.05)])
    g2 = synth.genome(77, 10000, [(500, 3, 0.05)])
    assert np.array_equal(g1, g2) and g1.size == 11500
    r1, o1 = synth.reads(g1, 3000, 150, err_rate=0.01, n_rate=0.01, seed=4, threads=1)
    r2, o2 = synth.reads(g1, 3000, 150, err_rate=0.01, n_rate=0.01, seed=4, threads=7)
    assert np.array_equal(r1, r2) and np.array_equal(o1, o2)
    assert set(np.unique(r1).tolist()) <= set(b"ACGTN")


@pytest.mark.parametrize("k", [3, 21, 31, 55, 100])
def test_range_slices_concatenate_to_the_full_count(k):
    """Slices over a partition of the top key bits, taken in order, are the
    full histogram; every key of a slice has its top bits in the slice's range
    (read off the key as a Python int)."""
    text, offs = synth.ragged_reads(4242 + k, 300, 0, 2 * k + 60, b"ACGTACGTacgtN")
    full_k, full_c = oracle.count(text, offs, k, threads=2)
    bits = min(2 * k, 6)
    cuts = [0, 1, 5, 17, 18, 40, 2 ** bits]
    ks, cs = [], []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        sk, sc = oracle.count_range(text, offs, k, bits, lo, hi, threads=3)
        for key in keys_as_ints(sk, k):
            assert lo <= key >> (2 * k - bits) < hi
        ks.append(sk)
        cs.append(sc)
    assert np.array_equal(np.concatenate(ks), full_k)
    assert np.array_equal(np.concatenate(cs), full_c)
    # an empty range gives nothing
    ek, ec = oracle.count_range(text, offs, k, bits, 7, 7)
    assert ek.shape[0] == 0 and ec.size == 0


def test_range_against_brute_force():
    text, offs = synth.ragged_reads(99, 60, 0, 50, b"ACGTacgtN")
    k = 5
    want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
    for lo, hi in ((0, 300), (300, 700), (700, 1024)):  # top 10 bits = the whole key
        sk, sc = oracle.count_range(text, offs, k, 10, lo, hi)
        assert _pairs(sk, sc, k) == [(x, c) for x, c in want if lo <= x < hi]
