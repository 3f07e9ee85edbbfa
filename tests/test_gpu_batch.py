"""Batched counting (one graph replay for many read sets) against the oracle
and against one plain call per set. Integer work: bit-exact."""
import numpy as np
import pytest

import oracle
import paper_2505_04431_amd as kc
import synth
from gpu_util import assert_same, gpu_count, to_device

pytestmark = pytest.mark.gpu


def make_batch(seed, n_sets, ks, min_g=300, max_g=30000, cov=5, read_len=100, empty_every=0):
    """Sets with their own genomes; returns concatenated reads/offsets and per-set data."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts, offs_all, set_reads, set_bytes, kk, per_set = [], [np.uint64(0)], [], [], [], []
    base = 0
    for s in range(n_sets):
        k = int(ks[s % len(ks)])
        if empty_every and s % empty_every == 0:
            r, o = np.zeros(0, np.uint8), np.zeros(1, np.uint64)
        else:
            G = int(np.exp(rng.uniform(np.log(min_g), np.log(max_g))))
            g = synth.genome(seed * 10007 + s, G)
            nr = max(1, G * cov // read_len)
            r, o = synth.reads(g, nr, read_len, err_rate=0.005, n_rate=0.0005, seed=seed + s,
                               threads=4)
        parts.append(r)
        offs_all.extend((o[1:] + np.uint64(base)).tolist())
        base += r.size
        set_reads.append(o.size - 1)
        set_bytes.append(r.size)
        kk.append(k)
        per_set.append((r, o, k))
    reads = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    offsets = np.array(offs_all, dtype=np.uint64)
    return reads, offsets, set_reads, set_bytes, kk, per_set


def check_batch(plan, rt, ot, per_set, against="oracle"):
    keys, cnts, set_off = plan.run(rt, ot)
    keys = keys.cpu().numpy().view(np.uint64)
    cnts = cnts.cpu().numpy().view(np.uint32)
    assert set_off[-1] == keys.size
    for s, (r, o, k) in enumerate(per_set):
        a, b = int(set_off[s]), int(set_off[s + 1])
        got = (keys[a:b], cnts[a:b])
        want = oracle.count(r, o, k) if against == "oracle" else gpu_count(r, o, k, P=2)
        assert_same(got, want, "set %d (k=%d)" % (s, k))
    return keys, cnts, set_off


def test_batch_mixed_k_against_oracle_and_plain():
    reads, offsets, sr, sb, ks, per_set = make_batch(1, 37, [21, 31, 5, 32, 16, 1], empty_every=9)
    rt, ot = to_device(reads, offsets)
    plan = kc.BatchPlan(sr, sb, ks, P=4)
    check_batch(plan, rt, ot, per_set, "oracle")
    check_batch(plan, rt, ot, per_set, "plain")
    st = plan.stats()
    assert st["valid_windows"] == sum(oracle.valid_windows(r, o, k) for r, o, k in per_set)
    plan.close()


def test_batch_graph_replays_with_eager_work_between():
    import torch
    reads, offsets, sr, sb, ks, per_set = make_batch(2, 20, [21, 31])
    rt, ot = to_device(reads, offsets)
    plan = kc.BatchPlan(sr, sb, ks, P=1)
    cap = plan.max_outputs
    keys = torch.empty(cap, dtype=torch.int64, device=rt.device)
    cnts = torch.empty(cap, dtype=torch.int32, device=rt.device)
    ref = None
    for rep in range(4):
        keys.fill_(-1)
        n, set_off = plan.run_into(rt, ot, keys, cnts, cap)
        got = (keys[:n].cpu().numpy().copy(), cnts[:n].cpu().numpy().copy(), set_off.copy())
        # eager work on the device between replays
        gk, gc = gpu_count(*per_set[rep % len(per_set)][:2], 31)
        torch.cuda.synchronize()
        if ref is None:
            ref = got
            for s, (r, o, k) in enumerate(per_set):
                a, b = int(set_off[s]), int(set_off[s + 1])
                assert_same((got[0][a:b].view(np.uint64), got[1][a:b].view(np.uint32)),
                            oracle.count(r, o, k), "set %d" % s)
        else:
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
            assert np.array_equal(got[2], ref[2])
    # new output buffers: the graph is recorded again
    keys2 = torch.empty(cap, dtype=torch.int64, device=rt.device)
    cnts2 = torch.empty(cap, dtype=torch.int32, device=rt.device)
    n2, set_off2 = plan.run_into(rt, ot, keys2, cnts2, cap)
    assert n2 == ref[0].size and np.array_equal(set_off2, ref[2])
    assert np.array_equal(keys2[:n2].cpu().numpy(), ref[0])
    plan.close()


def test_batch_layout_mismatch_and_capacity():
    import torch
    reads, offsets, sr, sb, ks, per_set = make_batch(3, 6, [31])
    rt, ot = to_device(reads, offsets)
    bad = list(sb)
    bad[0] += 1
    bad[1] -= 1
    plan = kc.BatchPlan(sr, bad, ks)
    with pytest.raises(kc.KcError) as e:
        plan.run(rt, ot)
    assert e.value.status == -1
    plan.close()
    plan = kc.BatchPlan(sr, sb, ks)
    keys = torch.empty(10, dtype=torch.int64, device=rt.device)
    cnts = torch.empty(10, dtype=torch.int32, device=rt.device)
    with pytest.raises(kc.KcError) as e:
        plan.run_into(rt, ot, keys, cnts, 10)
    total = sum(len(oracle.count(r, o, k)[1]) for r, o, k in per_set)
    assert e.value.status == -3 and e.value.n_out == total
    plan.close()
    with pytest.raises(kc.KcError):
        kc.BatchPlan(sr, sb, [33] * len(ks))


def test_batch_many_sets_c4_shape_sample():
    """Sets sampled like the 4,096-set workload (log-uniform genome sizes, 20x,
    150 bp, 0.5% errors, k in {21, 31}) at a reduced size range."""
    reads, offsets, sr, sb, ks, per_set = make_batch(4, 300, [21, 31], min_g=2000, max_g=60000,
                                                     cov=20, read_len=150)
    rt, ot = to_device(reads, offsets)
    plan = kc.BatchPlan(sr, sb, ks, P=1)
    check_batch(plan, rt, ot, per_set, "plain")
    plan.close()


def test_batch_k32_single_set_class_and_forced_overflow():
    """A class of one k = 32 set (no set-id bits: the key is the whole word),
    and a plan whose leaves overflow (no split below huge leaf sizes), so that
    the per-set fallback counts the wave; both against the oracle."""
    reads, offsets, sr, sb, ks, per_set = make_batch(5, 4, [32, 21, 31, 21], min_g=5000,
                                                     max_g=20000)
    rt, ot = to_device(reads, offsets)
    print("batch: one k=32 set, default options", flush=True)
    plan = kc.BatchPlan(sr, sb, ks, P=2)
    assert any(w["n_classes"] >= 3 for w in plan.waves)
    check_batch(plan, rt, ot, per_set, "oracle")
    assert plan.stats()["n_overflow"] == 0
    plan.close()
    print("batch: forced overflow (leaf_attempt 2^30, 1024-slot tables)", flush=True)
    plan = kc.BatchPlan(sr, sb, ks, P=2,
                        opts=kc.options(leaf_attempt=1 << 30, table_slots_log2=10, shard_bits=1))
    check_batch(plan, rt, ot, per_set, "oracle")
    assert plan.stats()["n_overflow"] >= 1
    plan.close()


def test_batch_tuner_candidates_against_oracle():
    """Every option set the tuners try, on sets of k = 21 (one-word class keys)
    and k = 31 (two-word class keys, whose tables hold 2,048 slots: a leaf
    target of 8,192 records makes their leaves overflow, so the per-set
    fallback runs after the wave's graph), each against the oracle."""
    from paper_2505_04431_amd import tuner
    reads, offsets, sr, sb, ks, per_set = make_batch(8, 24, [21, 31], min_g=3000, max_g=60000,
                                                     cov=10, read_len=150)
    rt, ot = to_device(reads, offsets)
    want = [oracle.count(r, o, k) for r, o, k in per_set]
    cands = list(tuner.DEFAULT_CANDIDATES) + [{"split_tile": 8}, {"scatter_tile": 16,
                                                                  "leaf_target": 8192}]
    for opts in cands:
        print("batch: options %s" % opts, flush=True)
        plan = kc.BatchPlan(sr, sb, ks, P=1, opts=kc.options(**opts))
        for _ in range(2):  # record, then replay
            keys, cnts, set_off = plan.run(rt, ot)
            keys = keys.cpu().numpy().view(np.uint64)
            cnts = cnts.cpu().numpy().view(np.uint32)
            assert set_off[-1] == keys.size
            for s, (r, o, k) in enumerate(per_set):
                a, b = int(set_off[s]), int(set_off[s + 1])
                assert_same((keys[a:b], cnts[a:b]), want[s],
                            "options %s, set %d (k=%d)" % (opts, s, k))
        print("batch:   overflowed waves %d" % plan.stats()["n_overflow"], flush=True)
        plan.close()


def test_batch_memory_waves_from_a_budget():
    """A device budget cuts the sets into several waves; running all waves at
    once and each wave from its own inputs both give the oracle's counts."""
    import torch
    reads, offsets, sr, sb, ks, per_set = make_batch(6, 40, [21, 31], min_g=2000, max_g=40000,
                                                     cov=10)
    rt, ot = to_device(reads, offsets)
    one = kc.BatchPlan(sr, sb, ks, P=1)
    assert len(one.waves) == 1
    budget = one.waves[0]["device_bytes"] // 4
    one.close()
    plan = kc.BatchPlan(sr, sb, ks, P=1, hbm_budget=budget)
    print("batch: %d waves under a budget of %d bytes" % (len(plan.waves), budget), flush=True)
    assert len(plan.waves) >= 3
    assert all(w["device_bytes"] <= budget for w in plan.waves)
    assert sum(w["n_sets"] for w in plan.waves) == len(per_set)
    keys, cnts, set_off = check_batch(plan, rt, ot, per_set, "oracle")
    # wave by wave, each from a copy of only its reads
    for wi, w in enumerate(plan.waves):
        a, b = w["first_byte"], w["first_byte"] + w["n_bytes"]
        r0, nr = w["first_read"], w["n_reads"]
        wr = rt[a:b].clone()
        wo = (ot[r0:r0 + nr + 1] - a).clone()
        cap = max(1, int(b - a))
        kk = torch.empty(cap, dtype=torch.int64, device=rt.device)
        cc = torch.empty(cap, dtype=torch.int32, device=rt.device)
        n, so = plan.run_wave_into(wi, wr, wo, kk, cc, cap)
        s0 = w["first_set"]
        base = int(set_off[s0])
        assert n == int(set_off[s0 + w["n_sets"]]) - base
        assert np.array_equal(so, set_off[s0:s0 + w["n_sets"] + 1] - np.uint64(base))
        assert np.array_equal(kk[:n].cpu().numpy().view(np.uint64), keys[base:base + n])
        assert np.array_equal(cc[:n].cpu().numpy().view(np.uint32), cnts[base:base + n])
    plan.close()
    with pytest.raises(kc.KcError) as e:
        kc.BatchPlan(sr, sb, ks, P=1, hbm_budget=1 << 20)
    assert e.value.status == -2
