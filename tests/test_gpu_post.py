"""k-mer spectrum and minimum-count filtering of a count result, against the
result-use oracles (oracle/post.py) applied to the oracle's count."""
import numpy as np
import pytest

import oracle
from oracle import post
import paper_2505_04431_amd as kc
import synth
from gpu_util import assert_same, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def result():
    c = synth.make_config(2, frac=0.05)
    out = {}
    for k in (31, 55):
        want = oracle.count(c["reads"], c["offsets"], k)
        rt, ot = to_device(c["reads"], c["offsets"])
        keys, cnts = kc.count(rt, ot, k, P=8)
        out[k] = (keys, cnts, want)
    return out


@pytest.mark.parametrize("k", [31, 55])
@pytest.mark.parametrize("max_count", [1, 2, 7, 300, 5000])
def test_spectrum(result, k, max_count):
    keys, cnts, (wk, wc) = result[k]
    h = kc.spectrum(cnts, max_count)
    want = post.spectrum(wc, max_count)
    assert np.array_equal(h, want)
    assert int(h.sum()) == len(wc)


@pytest.mark.parametrize("k", [31, 55])
@pytest.mark.parametrize("min_count", [0, 1, 2, 3, 40, 10**9])
def test_filter_min_count(result, k, min_count):
    keys, cnts, (wk, wc) = result[k]
    fk, fc = kc.filter_min_count(keys, cnts, k, min_count)
    got = (fk.cpu().numpy().view(np.uint64), fc.cpu().numpy().view(np.uint32))
    assert_same(got, post.filter_min_count(wk, wc, min_count), "min_count %d" % min_count)


def test_post_errors_and_empty():
    import torch
    dev = torch.device("cuda:0")
    e = torch.empty(0, dtype=torch.int32, device=dev)
    ek = torch.empty(0, dtype=torch.int64, device=dev)
    assert kc.spectrum(e, 5).sum() == 0
    fk, fc = kc.filter_min_count(ek, e, 31, 2)
    assert fk.numel() == 0 and fc.numel() == 0
    with pytest.raises(kc.KcError):
        kc.spectrum(e, 0)
    with pytest.raises(kc.KcError):
        kc.filter_min_count(ek, e, 0, 2)
