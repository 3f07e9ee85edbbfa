"""Shared helpers for GPU tests: run the HIP path through the C ABI on numpy inputs."""
from __future__ import annotations

import numpy as np

import paper_2505_04431_amd as kc


def device():
    import torch
    return torch.device("cuda:0")


def to_device(reads: np.ndarray, offsets: np.ndarray, pad_front: int = 0):
    """Copy inputs to the GPU; pad_front > 0 shifts the reads inside the buffer
    (offsets[0] = pad_front) so the unaligned path and a nonzero base are used."""
    import torch
    dev = device()
    if pad_front:
        buf = np.concatenate([np.full(pad_front, ord("N"), dtype=np.uint8), reads])
        offs = offsets + np.uint64(pad_front)
    else:
        buf, offs = reads, offsets
    if buf.size == 0:
        buf = np.zeros(1, dtype=np.uint8)
    rt = torch.from_numpy(np.ascontiguousarray(buf)).to(dev)
    ot = torch.from_numpy(np.ascontiguousarray(offs).view(np.int64)).to(dev)
    return rt, ot


def gpu_count(reads, offsets, k, P=1, pad_front=0, **opts):
    rt, ot = to_device(reads, offsets, pad_front)
    o = kc.options(**opts) if opts else None
    keys, cnt = kc.count(rt, ot, k, P, opts=o)
    return keys.cpu().numpy().view(np.uint64), cnt.cpu().numpy().view(np.uint32)


def assert_same(got, want, what=""):
    gk, gc = got
    wk, wc = want
    assert gk.shape == wk.shape, "%s: %s keys vs %s expected" % (what, gk.shape, wk.shape)
    if not np.array_equal(gk, wk):
        i = int(np.flatnonzero((gk != wk).reshape(len(gk), -1).any(axis=1))[0])
        raise AssertionError("%s: first key mismatch at %d: %s vs %s" % (what, i, gk[i], wk[i]))
    if not np.array_equal(gc, wc):
        i = int(np.flatnonzero(gc != wc)[0])
        raise AssertionError("%s: first count mismatch at %d (key %s): %d vs %d"
                             % (what, i, gk[i], gc[i], wc[i]))
