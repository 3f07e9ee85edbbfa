"""Full-size parity on the largest single-GPU workload: 200 Mbp genome (110
Mbp uniform plus 90 Mbp of 50 repeat families with Zipf(1.2) copy numbers),
40,000,000 reads of 150 bp at 30x, k = 31 and k = 21, P = 256.

The oracle cannot sort 4.8e9 windows in test time, so this checks what it can
compute one by one at full size: the counts of sampled output keys and of
every key of sampled reads (oracle selected-key count over all reads), the
number of valid windows against the sum of counts, and the device self-check
(strictly increasing, canonical, in range)."""
import numpy as np
import pytest

import oracle
import paper_2505_04431_amd as kc
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    cfg = synth.make_config(3)
    return cfg


@pytest.mark.parametrize("k", [31, 21])
def test_config3_full_sampled(c3, k):
    import torch
    reads, offs = c3["reads"], c3["offsets"]
    dev = torch.device("cuda:0")
    print("c3 k=%d: %d reads, %d bytes" % (k, offs.size - 1, reads.size), flush=True)
    rt = torch.from_numpy(reads).to(dev)
    ot = torch.from_numpy(offs.view(np.int64)).to(dev)
    cap = kc.max_outputs(offs, k)
    keys = torch.empty(cap, dtype=torch.int64, device=dev)
    cnts = torch.empty(cap, dtype=torch.int32, device=dev)
    n = kc.count_into(rt, ot, k, c3["P"], keys, cnts, cap,
                      kc.options(check=1))
    st = kc.last_stats()
    del rt, ot
    W = oracle.valid_windows(reads, offs, k)
    assert st["valid_windows"] == W and st["distinct"] == n
    total = int(cnts[:n].to(torch.int64).sum().item())
    assert total == W
    rng = np.random.Generator(np.random.PCG64(0xC3 + k))
    # sampled output entries, spread over the whole key range
    idx = np.sort(rng.choice(n, size=3000, replace=False))
    it = torch.from_numpy(idx.astype(np.int64)).to(dev)
    sk = keys[it].cpu().numpy().view(np.uint64)
    sc = cnts[it].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(oracle.count_selected(reads, offs, k, sk), sc)
    # every key of sampled reads is present with its full-input count
    ridx = rng.choice(offs.size - 1, size=40, replace=False)
    parts = [reads[int(offs[i]):int(offs[i + 1])] for i in ridx]
    po = np.zeros(len(parts) + 1, dtype=np.uint64)
    np.cumsum([p.size for p in parts], out=po[1:])
    rk, _ = oracle.count(np.concatenate(parts), po, k)
    rkt = torch.from_numpy(rk.view(np.int64)).to(dev)
    pos = torch.searchsorted(keys[:n], rkt)  # keys are < 2^62: signed order is key order
    assert int(pos.max().item()) < n
    found = keys[pos].cpu().numpy().view(np.uint64)
    assert np.array_equal(found, rk)
    gc = cnts[pos].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(oracle.count_selected(reads, offs, k, rk), gc)
    del keys, cnts
    kc.lib().kc_release_scratch()
    torch.cuda.empty_cache()
