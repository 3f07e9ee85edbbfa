"""The allocation-free entry point (kc_count_noalloc) against the allocating
one (kc_count_ex) on the same inputs: element-wise equal results on calls in
a row, the later ones smaller, so that stale contents of the shared fixed
scratch would show; an input larger than the scratch is refused with a clear
error and the next call still works."""
import numpy as np
import pytest

import paper_2505_04431_amd as kc
import synth
from gpu_util import assert_same, to_device
from paper_2505_04431_amd.kc import key_words

pytestmark = pytest.mark.gpu


def _both(reads, offs, k, P, pad_front=0, **opts):
    import torch
    rt, ot = to_device(reads, offs, pad_front)
    words = key_words(k)
    cap = max(1, kc.max_outputs(offs, k))
    shape = (cap, words) if words > 1 else (cap,)
    o = kc.options(**opts) if opts else None
    k1 = torch.empty(shape, dtype=torch.int64, device=rt.device)
    c1 = torch.empty(cap, dtype=torch.int32, device=rt.device)
    n1 = kc.count_into(rt, ot, k, P, k1, c1, cap, o)
    k2 = torch.full(shape, -1, dtype=torch.int64, device=rt.device)
    c2 = torch.full((cap,), -1, dtype=torch.int32, device=rt.device)
    n2 = kc.count_noalloc_into(rt, ot, k, P, k2, c2, cap, o)
    torch.cuda.synchronize()
    got = (k2[:n2].cpu().numpy().view(np.uint64), c2[:n2].cpu().numpy().view(np.uint32))
    want = (k1[:n1].cpu().numpy().view(np.uint64), c1[:n1].cpu().numpy().view(np.uint32))
    return got, want


@pytest.mark.parametrize("k", [31, 55])
def test_noalloc_equals_allocating_calls_in_a_row(k):
    print("noalloc k=%d: workload 1 full, then workload 2 at 0.3%%, then ragged reads" % k,
          flush=True)
    c1 = synth.make_config(1)
    c2 = synth.make_config(2, frac=0.003)
    rr, ro = synth.ragged_reads(5, 300, 0, 400)
    for name, (r, o), P, pad in (("workload 1", (c1["reads"], c1["offsets"]), 1, 0),
                                 ("workload 2 (0.3%)", (c2["reads"], c2["offsets"]), 64, 3),
                                 ("ragged", (rr, ro), 5, 1)):
        got, want = _both(r, o, k, P, pad_front=pad, check=1)
        assert len(want[1]) > 0
        assert_same(got, want, "%s k=%d" % (name, k))


def test_noalloc_refinement_and_limit():
    import torch
    print("noalloc: refinement case, then an input beyond the fixed scratch", flush=True)
    c = synth.make_config(2, frac=0.02)
    # leaves that overflow their tables: the refinement carves its buffers too
    got, want = _both(c["reads"], c["offsets"], 31, 7, shard_bits=6, leaf_target=30_000,
                      leaf_attempt=40_000)
    assert_same(got, want, "refinement")
    # 16 MB of reads at k = 31 need more than the fixed scratch: refused before any launch
    n = 16 << 20
    rt = torch.full((n,), ord("A"), dtype=torch.uint8, device="cuda:0")
    ot = torch.tensor([0, n], dtype=torch.int64, device="cuda:0")
    ko = torch.empty(16, dtype=torch.int64, device="cuda:0")
    co = torch.empty(16, dtype=torch.int32, device="cuda:0")
    with pytest.raises(kc.KcError) as e:
        kc.count_noalloc_into(rt, ot, 31, 1, ko, co, 16)
    assert e.value.status == -2 and "fixed scratch" in str(e.value)
    # a smaller call right after works and matches
    c1 = synth.make_config(1, frac=0.3)
    got, want = _both(c1["reads"], c1["offsets"], 31, 1)
    assert_same(got, want, "after the refusal")
