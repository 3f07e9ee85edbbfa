"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Integer work: every comparison is bit-exact, element by element.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same, gpu_count, to_device
from helpers import keys_as_ints, revcomp_bytes, to_arrays
from oracle import brute

pytestmark = pytest.mark.gpu

KS = [1, 2, 3, 4, 5, 8, 15, 16, 17, 21, 31, 32, 33, 55, 63, 64]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _pairs(keys, cnt, k):
    return list(zip(keys_as_ints(keys, k), [int(c) for c in cnt]))


def test_hand_examples():
    for e in json.load(open(GOLDEN))["examples"]:
        r, o = to_arrays(e["reads"])
        keys, cnt = gpu_count(r, o, e["k"], P=2, check=1)
        assert _pairs(keys, cnt, e["k"]) == [(brute.encode(s), c) for s, c in e["expect"]], e["name"]


@pytest.mark.parametrize("k", KS)
def test_brute_force_ragged(k):
    for seed in range(2):
        text, offs = synth.ragged_reads(1000 * k + seed, 60, 0, 3 * k + 40, b"ACGTACGTACGTacgtNR")
        want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
        keys, cnt = gpu_count(text, offs, k, P=3, check=1)
        assert _pairs(keys, cnt, k) == want


@pytest.mark.parametrize("k", [1, 2, 7, 16, 21, 31, 32, 33, 47, 55, 63, 64])
def test_oracle_random_genome_reads(k):
    # several thousand reads: many shards, several tiles per shard, ragged tail
    g = synth.genome(500 + k, 40_000, [(800, 10, 0.02)])
    r, o = synth.reads(g, 3001, 151, err_rate=0.01, n_rate=0.002, seed=k)
    assert_same(gpu_count(r, o, k, P=5, check=1), oracle.count(r, o, k), "k=%d" % k)


def test_config1_full_element_wise():
    c = synth.make_config(1)
    want = oracle.count(c["reads"], c["offsets"], 31)
    assert_same(gpu_count(c["reads"], c["offsets"], 31, P=1, check=1), want, "config 1")


@pytest.mark.parametrize("P", [1, 2, 3, 64, 256, 1024])
def test_p_invariance(P):
    c = synth.make_config(2, frac=0.05)
    want = oracle.count(c["reads"], c["offsets"], 31)
    assert_same(gpu_count(c["reads"], c["offsets"], 31, P=P), want, "P=%d" % P)


@pytest.mark.parametrize("opts", [
    dict(table_slots_log2=10),
    dict(table_slots_log2=11, leaf_target=300),          # deep splits
    dict(leaf_attempt=1 << 30),                           # overflow -> split path
    dict(shard_bits=1),
    dict(shard_bits=10, leaf_target=64, leaf_attempt=128),
    # split and unsplit shards whose leaves overflow: refinement from both buffers
    dict(shard_bits=6, leaf_target=30_000, leaf_attempt=40_000),
    dict(shard_bits=6, leaf_target=30_000, leaf_attempt=40_000, refine_bits=7),
    # 16,384-record LDS tiles in the owner and the split scatter
    dict(scatter_tile=16, split_tile=16),
    dict(scatter_tile=16, split_tile=8, shard_bits=10, leaf_target=64, leaf_attempt=128),
    dict(scatter_tile=8, split_tile=16, table_slots_log2=11, leaf_target=300),
    dict(preagg=2), dict(preagg=2, mode=1), dict(split_tile=8, preagg=1),
])
def test_knob_invariance(opts):
    c = synth.make_config(2, frac=0.02)
    for k in (31, 55):
        want = oracle.count(c["reads"], c["offsets"], k)
        assert_same(gpu_count(c["reads"], c["offsets"], k, P=7, check=1, **opts), want,
                    "k=%d %s" % (k, opts))


def test_fast_path_and_recursive_fallback_agree():
    """Default settings finish in the device-planned path; huge unsplit leaves
    overflow their tables and only those are partitioned further."""
    import paper_2505_04431_amd as kc
    c = synth.make_config(2, frac=0.05)
    want = oracle.count(c["reads"], c["offsets"], 31)
    assert_same(gpu_count(c["reads"], c["offsets"], 31, P=64), want, "fast path")
    st = kc.last_stats()
    assert st["n_overflow"] == 0 and st["n_levels"] == 1
    assert st["valid_windows"] == int(want[1].sum()) and st["distinct"] == len(want[1])
    assert_same(gpu_count(c["reads"], c["offsets"], 31, P=64, leaf_attempt=1 << 30,
                          shard_bits=4), want, "fallback path")
    st = kc.last_stats()
    assert st["n_overflow"] >= 1


def test_refinement_settles_frequent_keys():
    """One k-mer with 200,000 copies next to many distinct ones in a leaf that
    overflows: the part holding the frequent key is counted whole."""
    import paper_2505_04431_amd as kc
    rnd, ro = synth.ragged_reads(77, 600, 100, 200)
    reads = np.concatenate([np.full(200_030, ord("A"), np.uint8), rnd])
    offs = np.concatenate([[0], ro + np.uint64(200_030)]).astype(np.uint64)
    want = oracle.count(reads, offs, 31)
    for k, opts in ((31, dict(shard_bits=1, leaf_attempt=1 << 30, table_slots_log2=10)),
                    (55, dict(shard_bits=2, leaf_attempt=1 << 30, table_slots_log2=10))):
        w = want if k == 31 else oracle.count(reads, offs, k)
        assert_same(gpu_count(reads, offs, k, check=1, **opts), w, "k=%d" % k)
        st = kc.last_stats()
        assert st["n_overflow"] >= 1 and st["max_leaf_windows"] >= 200_030 - k + 1


def test_strand_flip_permutation_and_unaligned_base():
    g = synth.genome(31, 30_000, [(500, 20, 0.01)])
    r, o = synth.reads(g, 2000, 150, err_rate=0.005, n_rate=0.001, seed=3)
    base = gpu_count(r, o, 31, P=4)
    assert_same(gpu_count(revcomp_bytes(r, o), o, 31, P=4), base, "strand flip")
    perm = np.random.Generator(np.random.PCG64(1)).permutation(o.size - 1)
    chunks = [r[int(o[i]):int(o[i + 1])] for i in perm]
    o2 = np.zeros_like(o)
    np.cumsum([len(x) for x in chunks], out=o2[1:])
    assert_same(gpu_count(np.concatenate(chunks), o2, 31, P=4), base, "permutation")
    for pad in (1, 3, 13, 64, 77):
        assert_same(gpu_count(r, o, 31, P=4, pad_front=pad), base, "pad %d" % pad)


def test_empty_and_degenerate_inputs():
    empty = (np.zeros(0, dtype=np.uint8), np.zeros(1, dtype=np.uint64))
    k, c = gpu_count(*empty, 31)
    assert k.size == 0 and c.size == 0
    r, o = to_arrays(["", "ACG", "", "NNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNN"])
    k, c = gpu_count(r, o, 31)
    assert k.size == 0
    r, o = to_arrays(["A" * 5000, "T" * 3000])
    k, c = gpu_count(r, o, 31, check=1)
    assert k.tolist() == [0] and c.tolist() == [5000 - 30 + 3000 - 30]
    r, o = to_arrays(["ACGT" * 2000])
    for kk in (1, 2, 64):
        assert_same(gpu_count(r, o, kk), oracle.count(r, o, kk), "periodic k=%d" % kk)


def test_error_paths():
    import torch
    import paper_2505_04431_amd as kc
    r, o = to_arrays(["ACGTACGT"])
    rt, ot = to_device(r, o)
    keys = torch.empty(8, dtype=torch.int64, device=rt.device)
    cnt = torch.empty(8, dtype=torch.int32, device=rt.device)
    for bad_k in (0, 129):
        with pytest.raises(kc.KcError) as e:
            kc.count_into(rt, ot, bad_k, 1, keys, cnt, 8)
        assert e.value.status == -1
    with pytest.raises(kc.KcError) as e:
        kc.count_into(rt, ot, 3, 0, keys, cnt, 8)
    assert e.value.status == -1
    want = oracle.count(r, o, 2)
    with pytest.raises(kc.KcError) as e:
        kc.count_into(rt, ot, 2, 1, keys, cnt, len(want[0]) - 1)
    assert e.value.status == -3 and e.value.n_out == len(want[0])
    bad = torch.tensor([0, 5, 3], dtype=torch.int64, device=rt.device)
    with pytest.raises(kc.KcError) as e:
        kc.count_into(rt, bad, 2, 1, keys, cnt, 8)
    assert e.value.status == -1


def test_output_tensors_too_small_are_refused():
    """The binding refuses output tensors that cannot hold `capacity` keys of
    the key width (the library itself only sees raw pointers)."""
    import torch
    import paper_2505_04431_amd as kc
    r, o = to_arrays(["ACGTACGTACGTTTGCA" * 8])
    rt, ot = to_device(r, o)
    dev = rt.device
    for k, words in ((31, 1), (55, 2), (100, 4)):
        short_keys = torch.empty(8 * words - 1, dtype=torch.int64, device=dev)
        cnt = torch.empty(8, dtype=torch.int32, device=dev)
        with pytest.raises(ValueError):
            kc.count_into(rt, ot, k, 1, short_keys, cnt, 8)
        with pytest.raises(ValueError):
            kc.count_noalloc_into(rt, ot, k, 1, short_keys, cnt, 8)
        keys = torch.empty(8 * words, dtype=torch.int64, device=dev)
        with pytest.raises(ValueError):
            kc.count_into(rt, ot, k, 1, keys, cnt[:7], 8)


def test_config2_full_element_wise():
    """The benchmark workload (5 Mbp + repeats, 1M reads, k=31, P=64), full size."""
    c = synth.make_config(2)
    want = oracle.count(c["reads"], c["offsets"], 31)
    got = gpu_count(c["reads"], c["offsets"], 31, P=64, check=1)
    assert_same(got, want, "config 2")
    assert int(got[1].sum(dtype=np.uint64)) == oracle.valid_windows(c["reads"], c["offsets"], 31)


def test_k55_long_reads():
    g = synth.genome(55, 200_000, [(3000, 5, 0.01)])
    r, o = synth.reads(g, 300, 10_000, err_rate=0.01, seed=5)
    assert_same(gpu_count(r, o, 55, P=8, check=1), oracle.count(r, o, 55), "k=55 long reads")


def test_count_beyond_32_bits_is_reported():
    """A k-mer seen 2^32 + 1 times: the call fails with KC_E_OVERFLOW instead of
    returning a wrapped count."""
    import torch
    import paper_2505_04431_amd as kc
    n = (1 << 32) + 31  # k = 31: 2^32 + 1 windows, all the same key
    dev = torch.device("cuda:0")
    rt = torch.full((n,), ord("A"), dtype=torch.uint8, device=dev)
    ot = torch.tensor([0, n], dtype=torch.int64, device=dev)
    keys = torch.empty(16, dtype=torch.int64, device=dev)
    cnts = torch.empty(16, dtype=torch.int32, device=dev)
    with pytest.raises(kc.KcError) as e:
        kc.count_into(rt, ot, 31, 1, keys, cnts, 16)
    assert e.value.status == -4
    del rt
    kc.lib().kc_release_scratch()
    torch.cuda.empty_cache()


# ---- sort-based leaf count (mode 1): the same results

@pytest.mark.parametrize("k", [1, 5, 16, 31, 32, 33, 55, 64])
def test_sort_mode_brute_force(k):
    text, offs = synth.ragged_reads(7000 + k, 80, 0, 3 * k + 40, b"ACGTACGTACGTacgtNR")
    want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
    keys, cnt = gpu_count(text, offs, k, P=3, check=1, mode=1)
    assert _pairs(keys, cnt, k) == want


@pytest.mark.parametrize("opts", [
    dict(mode=1),
    dict(mode=1, leaf_target=20_000, leaf_attempt=20_000),  # leaves too big to sort: refined
    dict(mode=1, shard_bits=10, leaf_target=64, leaf_attempt=128),
])
def test_sort_mode_options(opts):
    c = synth.make_config(2, frac=0.02)
    for k in (31, 55):
        want = oracle.count(c["reads"], c["offsets"], k)
        assert_same(gpu_count(c["reads"], c["offsets"], k, P=7, check=1, **opts), want,
                    "k=%d %s" % (k, opts))


def test_sort_mode_single_key_leaves_and_full_size():
    import paper_2505_04431_amd as kc
    rnd, ro = synth.ragged_reads(78, 600, 100, 200)
    reads = np.concatenate([np.full(200_030, ord("A"), np.uint8), rnd])
    offs = np.concatenate([[0], ro + np.uint64(200_030)]).astype(np.uint64)
    for k in (31, 55):
        assert_same(gpu_count(reads, offs, k, check=1, mode=1), oracle.count(reads, offs, k),
                    "frequent key k=%d" % k)
    c = synth.make_config(2)
    assert_same(gpu_count(c["reads"], c["offsets"], 31, P=64, check=1, mode=1),
                oracle.count(c["reads"], c["offsets"], 31), "config 2, mode 1")
    st = kc.last_stats()
    assert st["distinct"] > 0


def test_calls_on_two_streams_in_a_row():
    """A call returns with its last kernels (the copy into the outputs) still
    queued on its stream; the next call of the same thread on another stream
    reuses the thread's device buffers and must not overwrite them early."""
    import torch
    import paper_2505_04431_amd as kc
    a = synth.make_config(2, frac=0.15)
    g = synth.genome(5, 300_000, [(2000, 8, 0.02)])
    br, bo = synth.reads(g, 60_000, 150, err_rate=0.01, seed=6)
    ra, oa = to_device(a["reads"], a["offsets"])
    rb, ob = to_device(br, bo)
    want_a = oracle.count(a["reads"], a["offsets"], 31)
    want_b = oracle.count(br, bo, 31)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            ka, ca = kc.count(ra, oa, 31, P=16)
        with torch.cuda.stream(s2):
            kb, cb = kc.count(rb, ob, 31, P=16)
        torch.cuda.synchronize()
        assert_same((ka.cpu().numpy().view(np.uint64), ca.cpu().numpy().view(np.uint32)), want_a,
                    "first call, stream 1")
        assert_same((kb.cpu().numpy().view(np.uint64), cb.cpu().numpy().view(np.uint32)), want_b,
                    "second call, stream 2")
    # the arena handed back (its blocks returned to the device) and grown again
    kc.lib().kc_release_scratch()
    with torch.cuda.stream(s2):
        ka, ca = kc.count(ra, oa, 31, P=16)
    torch.cuda.synchronize()
    assert_same((ka.cpu().numpy().view(np.uint64), ca.cpu().numpy().view(np.uint32)), want_a,
                "after release")


def test_arena_of_an_ended_thread():
    """A thread that counted and ended leaves its arena behind; the next count
    (on another thread) frees it and its own result is unaffected."""
    import threading
    import torch
    import paper_2505_04431_amd as kc
    g = synth.genome(9, 200_000, [(1500, 6, 0.02)])
    r, o = synth.reads(g, 40_000, 150, err_rate=0.01, seed=2)
    rt, ot = to_device(r, o)
    want = oracle.count(r, o, 55)
    got = {}

    def worker():
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            k1, c1 = kc.count(rt, ot, 55, P=8)
        s.synchronize()
        got["t"] = (k1.cpu().numpy().view(np.uint64), c1.cpu().numpy().view(np.uint32))

    for _ in range(2):
        th = threading.Thread(target=worker)
        th.start()
        th.join()
        assert_same(got["t"], want, "ended thread")
        k2, c2 = kc.count(rt, ot, 55, P=8)
        assert_same((k2.cpu().numpy().view(np.uint64), c2.cpu().numpy().view(np.uint32)), want,
                    "after the thread ended")


def test_arena_regrowth_sizes():
    """Inputs of rising and falling sizes on one thread: the arena grows
    stream-ordered from the device pool (by half its size at least), is kept
    when a smaller input follows, and is rebuilt after a release."""
    import paper_2505_04431_amd as kc
    g = synth.genome(13, 400_000, [(2000, 5, 0.02)])
    for i, n in enumerate((300, 4_000, 1_500, 30_000, 90_000, 20_000, 60_000)):
        r, o = synth.reads(g, n, 150, err_rate=0.01, seed=100 + n)
        k = 31 if i % 2 == 0 else 55
        assert_same(gpu_count(r, o, k, P=8), oracle.count(r, o, k), "n=%d k=%d" % (n, k))
        if i == 4:
            kc.lib().kc_release_scratch()


@pytest.mark.parametrize("k", [31, 21, 27])
def test_preaggregation_on_off_and_sort_mode(k):
    """Equal keys merged in the split scatter (records carrying counts) give
    the same histogram as plain records, through the hash-table leaves, the
    radix-sorted leaves and the refinement of overflowed leaves; on an input
    with heavy repeats the leaves read fewer records than there are windows."""
    import paper_2505_04431_amd as kc
    print("preagg k=%d: a 60 kbp genome with a 3 kbp family in 300 exact copies" % k, flush=True)
    g = synth.genome(4711, 60_000, [(3000, 300, 0.0)])
    reads, offs = synth.reads(g, 60_000, 150, err_rate=0.002, n_rate=0.0, seed=9)
    want = oracle.count(reads, offs, k)
    runs = {}
    for name, opts in (("on", dict(preagg=1)), ("off", dict(preagg=2)),
                       ("on, sort mode", dict(preagg=1, mode=1)),
                       ("on, refined", dict(preagg=1, shard_bits=4, leaf_target=60_000,
                                            leaf_attempt=70_000, table_slots_log2=10)),
                       ("on, refined sort", dict(preagg=1, mode=1, shard_bits=4,
                                                 leaf_target=60_000, leaf_attempt=70_000))):
        assert_same(gpu_count(reads, offs, k, P=5, check=1, **opts), want, name)
        runs[name] = kc.last_stats()
    W = runs["off"]["valid_windows"]
    assert runs["on"]["large_records"] < 0.9 * W
    assert runs["off"]["large_records"] + 0.01 * W >= runs["on"]["large_records"]
