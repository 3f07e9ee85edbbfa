"""Full-size parity on the largest single-GPU workload: 200 Mbp genome (110
Mbp uniform plus 90 Mbp of 50 repeat families with Zipf(1.2) copy numbers),
40,000,000 reads of 150 bp at 30x, k = 31 and k = 21, P = 256.

Element-wise: the GPU output is cut into four slices by the top two bits of
the key, and each slice is compared pair by pair with the oracle's tally of
the keys in that slice (the oracle decodes only the windows whose key falls
in the slice, so each pass holds a quarter of the keys). The slices cover
the whole key space, so the number of distinct keys is compared too; the
number of valid windows is compared with the oracle's count of them."""
import numpy as np
import pytest

import oracle
import paper_2505_04431_amd as kc
import synth

pytestmark = pytest.mark.gpu

SLICE_BITS = 2


@pytest.fixture(scope="module")
def c3():
    return synth.make_config(3)


@pytest.mark.parametrize("k", [31, 21])
def test_config3_full_element_wise(c3, k):
    import torch
    reads, offs = c3["reads"], c3["offsets"]
    dev = torch.device("cuda:0")
    print("c3 k=%d: %d reads, %d bytes, P=%d" % (k, offs.size - 1, reads.size, c3["P"]),
          flush=True)
    rt = torch.from_numpy(reads).to(dev)
    ot = torch.from_numpy(offs.view(np.int64)).to(dev)
    cap = kc.max_outputs(offs, k)
    keys = torch.empty(cap, dtype=torch.int64, device=dev)
    cnts = torch.empty(cap, dtype=torch.int32, device=dev)
    n = kc.count_into(rt, ot, k, c3["P"], keys, cnts, cap, kc.options(check=1))
    st = kc.last_stats()
    del rt, ot
    torch.cuda.empty_cache()
    assert st["valid_windows"] == oracle.valid_windows(reads, offs, k)
    assert st["distinct"] == n
    # keys are below 2^62, so signed order is key order for searchsorted
    shift = 2 * k - SLICE_BITS
    bounds = torch.tensor([s << shift for s in range(2 ** SLICE_BITS)] + [1 << (2 * k)],
                          dtype=torch.int64, device=dev)
    cut = torch.searchsorted(keys[:n], bounds).cpu().tolist()
    assert cut[0] == 0 and cut[-1] == n
    for s in range(2 ** SLICE_BITS):
        a, b = cut[s], cut[s + 1]
        got_k = keys[a:b].cpu().numpy().view(np.uint64)
        got_c = cnts[a:b].cpu().numpy().view(np.uint32)
        want_k, want_c = oracle.count_range(reads, offs, k, SLICE_BITS, s, s + 1,
                                            capacity=2 * (b - a) + 1024)
        print("  slice %d: %d pairs (oracle %d)" % (s, b - a, want_c.size), flush=True)
        assert got_k.size == want_k.size, "slice %d: %d keys vs %d" % (s, got_k.size, want_k.size)
        assert np.array_equal(got_k, want_k), "slice %d keys differ" % s
        assert np.array_equal(got_c, want_c), "slice %d counts differ" % s
        del got_k, got_c, want_k, want_c
    del keys, cnts
    kc.lib().kc_release_scratch()
    torch.cuda.empty_cache()
