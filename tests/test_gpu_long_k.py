"""Keys of 65..128 bases (four 64-bit words per key) on the HIP path against the
oracle (itself pinned by the string brute force at these k): brute force over
ragged reads, reads of a repeat-rich genome over many shards and tiles, long
reads, leaves refined after overflow, a single key of a huge count, the
self-check, P-invariance, and the uses of a result (filter, merge, server)."""
import numpy as np
import pytest

import oracle
import paper_2505_04431_amd as kc
import synth
from gpu_util import assert_same, gpu_count, to_device
from helpers import keys_as_ints
from oracle import brute

pytestmark = pytest.mark.gpu

LONG_KS = [65, 66, 77, 96, 97, 100, 121, 127, 128]


def _pairs(keys, cnt, k):
    return list(zip(keys_as_ints(keys, k), [int(c) for c in cnt]))


@pytest.mark.parametrize("k", LONG_KS)
def test_brute_force_ragged(k):
    for seed in range(2):
        text, offs = synth.ragged_reads(9000 * k + seed, 60, 0, 3 * k + 40, b"ACGTACGTACGTacgtNR")
        want = brute.count_strings(brute.split_reads(text.tobytes(), offs), k)
        keys, cnt = gpu_count(text, offs, k, P=3, check=1)
        assert keys.shape[1:] == (4,)
        assert _pairs(keys, cnt, k) == want


@pytest.mark.parametrize("k", [65, 100, 128])
@pytest.mark.parametrize("P", [1, 64])
def test_genome_reads(k, P):
    g = synth.genome(700 + k, 60_000, [(900, 12, 0.02)])
    r, o = synth.reads(g, 4001, 250, err_rate=0.01, n_rate=0.002, seed=k)
    assert_same(gpu_count(r, o, k, P=P, check=1), oracle.count(r, o, k), "k=%d P=%d" % (k, P))


@pytest.mark.parametrize("k", [70, 127])
def test_long_reads_unaligned(k):
    g = synth.genome(31 + k, 200_000, [(3000, 6, 0.03)])
    lens = np.random.Generator(np.random.PCG64(k)).integers(0, 6000, size=300).astype(np.uint64)
    r, o = synth.reads(g, 300, lens=lens, err_rate=0.005, n_rate=0.0005, seed=3)
    want = oracle.count(r, o, k)
    assert_same(gpu_count(r, o, k, P=5, check=1), want, "k=%d" % k)
    assert_same(gpu_count(r, o, k, P=5, pad_front=11), want, "k=%d unaligned" % k)


@pytest.mark.parametrize("opts", [
    dict(),
    dict(leaf_target=20_000, leaf_attempt=20_000),  # leaves too big to sort: refined
    dict(shard_bits=10, leaf_target=64, leaf_attempt=128),
    dict(mode=1, shard_bits=1),
])
def test_options_and_refinement(opts):
    c = synth.make_config(2, frac=0.02)
    for k in (80, 128):
        want = oracle.count(c["reads"], c["offsets"], k)
        assert_same(gpu_count(c["reads"], c["offsets"], k, P=7, check=1, **opts), want,
                    "k=%d %s" % (k, opts))


def test_frequent_key_and_its_neighbours():
    # one key of ~200,000 copies (a homopolymer run), plus reads that differ
    # from it in one base: a leaf far above the sort limit, refined down to the
    # single key
    rnd, ro = synth.ragged_reads(91, 400, 130, 260)
    run = np.full(200_030, ord("A"), np.uint8)
    near = np.full(130, ord("A"), np.uint8)
    near[-1] = ord("C")
    reads = np.concatenate([run, np.tile(near, 50), rnd])
    offs = np.concatenate([[0, 200_030], 200_030 + 130 * np.arange(1, 51),
                           200_030 + 130 * 50 + ro[1:].astype(np.int64)]).astype(np.uint64)
    for k in (65, 128):
        assert_same(gpu_count(reads, offs, k, check=1), oracle.count(reads, offs, k),
                    "frequent key k=%d" % k)


def test_uses_of_a_long_key_result():
    c = synth.make_config(2, frac=0.02)
    reads, offs = c["reads"], c["offsets"]
    k = 99
    want_k, want_c = oracle.count(reads, offs, k)
    rt, ot = to_device(reads, offs)
    keys, cnts = kc.count(rt, ot, k, P=8)
    # filter
    fk, fc = kc.filter_min_count(keys, cnts, k, 3)
    keep = want_c >= 3
    assert_same((fk.cpu().numpy().view(np.uint64), fc.cpu().numpy().view(np.uint32)),
                (want_k[keep], want_c[keep]), "filter")
    # spectrum
    h = kc.spectrum(cnts, 50)
    ref = np.zeros(51, np.uint64)
    np.add.at(ref, np.minimum(want_c.astype(np.int64), 50), 1)
    assert np.array_equal(h, ref)
    # merge of two halves = count of the whole
    n = offs.size - 1
    parts = []
    for r0, r1 in ((0, n // 2), (n // 2, n)):
        b0, b1 = int(offs[r0]), int(offs[r1])
        a, b = to_device(reads[b0:b1], offs[r0:r1 + 1] - np.uint64(b0))
        parts.append(kc.count(a, b, k, P=3))
    mk, mc = kc.merge_counts(parts[0][0], parts[0][1], parts[1][0], parts[1][1], k)
    assert_same((mk.cpu().numpy().view(np.uint64), mc.cpu().numpy().view(np.uint32)),
                (want_k, want_c), "merge")
    # the server
    srv = kc.Server(budget_bytes=8 << 30, workers=2)
    try:
        job = srv.submit(rt, ot, k, P=4)
        assert srv.wait(job) == "done", srv.info(job)
        sk, sc = srv.result(job)
        assert_same((sk.cpu().numpy().view(np.uint64), sc.cpu().numpy().view(np.uint32)),
                    (want_k, want_c), "server")
        srv.release(job)
    finally:
        srv.close()


def test_limits():
    r, o = synth.ragged_reads(5, 10, 100, 127)
    rt, ot = to_device(r, o)
    with pytest.raises(kc.KcError):
        kc.count(rt, ot, 129, P=1)
    assert kc.max_outputs(o, 128) == int(np.maximum(np.diff(o.astype(np.int64)) - 127, 0).sum())
    # reads all shorter than k: an empty result of the four-word shape
    keys, cnts = kc.count(rt, ot, 128, P=2)
    assert cnts.numel() == 0 and tuple(keys.shape) == (0, 4)
