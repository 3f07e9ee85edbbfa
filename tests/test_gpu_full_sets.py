"""Parity at the real sizes of the batched and served workloads (the scaled
versions live in test_gpu_batch.py / test_gpu_server.py): read sets and jobs
generated exactly as the 4,096-set and 10,000-job recipes make them, counted
through the batch plan and the server, each compared element by element with
the oracle on that set's or job's reads alone."""
import numpy as np
import pytest

import oracle
import paper_2505_04431_amd as kc
import synth
from gpu_util import assert_same, to_device

pytestmark = pytest.mark.gpu


def test_batch_real_size_sets_against_oracle():
    import torch
    spec = synth.c4_sets()
    rng = np.random.Generator(np.random.PCG64(0xC4F))
    small = [i for i, (g, _) in enumerate(spec) if g <= 1_000_000]
    large = [i for i, (g, _) in enumerate(spec) if g > 1_000_000]
    pick = sorted(rng.choice(small, size=24, replace=False).tolist() +
                  rng.choice(large, size=2, replace=False).tolist())
    # layout by (k, size) as the plan's classes expect contiguous byte ranges
    pick.sort(key=lambda i: (spec[i][1], -spec[i][0]))
    parts, offs, set_reads, set_bytes, ks, per = [], [np.zeros(1, np.uint64)], [], [], [], []
    base = 0
    for i in pick:
        r, o = synth.c4_set_reads(i, spec[i][0], threads=16)
        parts.append(r)
        offs.append(o[1:] + np.uint64(base))
        base += r.size
        set_reads.append(o.size - 1)
        set_bytes.append(r.size)
        ks.append(spec[i][1])
        per.append((r, o, spec[i][1]))
    print("sets %s, %d bytes" % (pick, base), flush=True)
    rt, ot = to_device(np.concatenate(parts), np.concatenate(offs))
    plan = kc.BatchPlan(set_reads, set_bytes, ks, P=1)
    keys, cnts, set_off = plan.run(rt, ot)
    torch.cuda.synchronize()
    hk, hc = keys.cpu().numpy().view(np.uint64), cnts.cpu().numpy().view(np.uint32)
    for s, (r, o, k) in enumerate(per):
        a, b = int(set_off[s]), int(set_off[s + 1])
        assert_same((hk[a:b], hc[a:b]), oracle.count(r, o, k), "set %d (k=%d, %d bytes)"
                    % (pick[s], k, r.size))
    plan.close()


def test_server_real_size_jobs_against_oracle():
    import torch
    specs = synth.c5_jobs()
    # jobs of up to 5 Mbp genomes, both read kinds and both k
    cand = [s for s in specs if s["genome_len"] <= 5_000_000]
    rng = np.random.Generator(np.random.PCG64(0xC5F))
    picks = []
    for want in ((150, 31), (150, 55), (10_000, 31), (10_000, 55)):
        c = [s for s in cand if (s["read_len"], s["k"]) == want]
        picks += [c[int(j)] for j in rng.choice(len(c), size=2, replace=False)]
    jobs = []
    for sp in picks:
        r, o = synth.c5_job_reads(sp, threads=16)
        jobs.append((r, o, sp["k"], sp["job"]))
    print("jobs %s" % [(j, k, r.size) for r, o, k, j in jobs], flush=True)
    dev_in = [to_device(r, o) for r, o, _, _ in jobs]
    torch.cuda.synchronize()
    srv = kc.Server(budget_bytes=96 << 30, workers=4)
    try:
        ids = [srv.submit(rt, ot, k, P=64) for (rt, ot), (_, _, k, _) in zip(dev_in, jobs)]
        for jid, (r, o, k, j) in zip(ids, jobs):
            assert srv.wait(jid) == "done"
            kk, cc = srv.result(jid)
            got = (kk.cpu().numpy().view(np.uint64), cc.cpu().numpy().view(np.uint32))
            assert_same(got, oracle.count(r, o, k), "job %d (k=%d, %d bytes)" % (j, k, r.size))
            srv.release(jid)
    finally:
        srv.close()
