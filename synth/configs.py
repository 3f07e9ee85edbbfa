"""The five workload recipes (genome, reads, k, P) with a size fraction.

``frac`` scales genome length and read count together (coverage kept), so that
the same recipe yields a small case for fast tests and the full-size case.
"""
from __future__ import annotations

import math

import numpy as np

from . import CONFIG_SEED_BASE, genome, reads

CONFIGS = {
    1: dict(name="c1_plain_k31_P1_100kbp_10x", backbone=100_000, families="none",
            n_reads=6_667, read_len=150, err=0.005, n_rate=0.0, ks=(31,), P=1),
    2: dict(name="c2_plain_k31_P64_5Mbp_repeats_30x", backbone=5_000_000, families="c2",
            n_reads=1_000_000, read_len=150, err=0.01, n_rate=1e-4, ks=(31,), P=64),
    3: dict(name="c3_plain_k31_k21_P256_200Mbp_zipf_30x", backbone=110_000_000, families="c3",
            n_reads=40_000_000, read_len=150, err=0.005, n_rate=0.0, ks=(31, 21), P=256),
}


def family_layout(kind: str, seed: int, frac: float = 1.0):
    """Repeat families as (length, copies, divergence) tuples."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0xFA11))
    if kind == "none":
        return []
    if kind == "c2":
        # 5 families of length U[1, 6] kbp, each inserted 40 times at 2% divergence.
        lens = rng.integers(1000, 6001, size=5)
        copies = max(1, int(round(40 * frac)))
        return [(int(l), copies, 0.02) for l in lens]
    if kind == "c3":
        # 50 families, length U[1, 6] kbp, Zipf(1.2) copy numbers capped at 1e4,
        # scaled so the copies total 90 Mbp (45% of 200 Mbp); divergence U[2, 5]%.
        lens = rng.integers(1000, 6001, size=50).astype(np.float64)
        divs = rng.uniform(0.02, 0.05, size=50)
        target = 90_000_000 * frac
        ranks = np.arange(1, 51, dtype=np.float64)
        cap = max(1.0, 1e4 * frac)

        def total(A):
            c = np.minimum(cap, np.round(A * ranks ** -1.2))
            return float((c * lens).sum())

        lo, hi = 0.0, 1e9
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if total(mid) < target:
                lo = mid
            else:
                hi = mid
        c = np.minimum(cap, np.round(hi * ranks ** -1.2)).astype(np.int64)
        return [(int(l), int(cc), float(d)) for l, cc, d in zip(lens, c, divs) if cc > 0]
    raise ValueError(kind)


def make_config(idx: int, frac: float = 1.0, threads: int | None = None):
    """Build config ``idx`` at size fraction ``frac``.

    Returns dict(reads=uint8[], offsets=uint64[n+1], ks=tuple, P=int, name=str, genome_len=int).
    """
    c = CONFIGS[idx]
    seed = CONFIG_SEED_BASE + idx
    backbone = max(1000, int(round(c["backbone"] * frac)))
    fams = family_layout(c["families"], seed, frac)
    g = genome(seed, backbone, fams)
    n_reads = max(1, int(round(c["n_reads"] * frac)))
    r, off = reads(g, n_reads, c["read_len"], err_rate=c["err"], n_rate=c["n_rate"],
                   seed=seed, threads=threads)
    name = c["name"] if frac == 1.0 else "%s@%g" % (c["name"], frac)
    return dict(reads=r, offsets=off, ks=c["ks"], P=c["P"], name=name, genome_len=int(g.shape[0]))


# ---- the batched workload: 4,096 independent read sets

def c4_sets(n_sets: int = 4096, seed: int = CONFIG_SEED_BASE + 4):
    """Per-set (genome length, k) of the batched workload: genome lengths
    log-uniform in [10 kbp, 10 Mbp], k drawn from {21, 31}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = np.exp(rng.uniform(math.log(1e4), math.log(1e7), size=n_sets)).astype(np.int64)
    ks = rng.choice(np.array([21, 31]), size=n_sets)
    return [(int(g), int(k)) for g, k in zip(G, ks)]


def c4_set_reads(s: int, genome_len: int, coverage: int = 20, read_len: int = 150,
                 err: float = 0.005, seed: int = CONFIG_SEED_BASE + 4, threads: int | None = None):
    """Reads of set s: its own uniform genome sampled at `coverage`."""
    g = genome(seed * 1000003 + s, genome_len)
    n = max(1, genome_len * coverage // read_len)
    return reads(g, n, read_len, err_rate=err, seed=seed + 17 * s + 1, threads=threads)


def c4_sample(n_sample: int, n_sets: int = 4096, seed: int = CONFIG_SEED_BASE + 4):
    """A seeded subset of the set indices (same size distribution)."""
    if n_sample >= n_sets:
        return list(range(n_sets))
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5A))
    return sorted(rng.choice(n_sets, size=n_sample, replace=False).tolist())


def waves(sizes, budget: int):
    """Greedy consecutive grouping of sizes into waves of at most `budget`."""
    out, cur, acc = [], [], 0
    for i, b in enumerate(sizes):
        if cur and acc + b > budget:
            out.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += b
    if cur:
        out.append(cur)
    return out


# ---- the served workload: a stream of independent counting jobs

def c5_jobs(n_jobs: int = 10_000, seed: int = CONFIG_SEED_BASE + 5):
    """Per-job recipe of the served workload: genome length log-uniform in
    [50 kbp, 50 Mbp] with 10% of it from repeat families, coverage U[10, 30],
    80% of jobs short reads (150 bp, 0.5% substitutions) and 20% long reads
    (10 kbp, 1% substitutions), k drawn from {31, 55}.

    Returns a list of dicts (job, genome_len, coverage, read_len, err, k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = np.exp(rng.uniform(math.log(5e4), math.log(5e7), size=n_jobs)).astype(np.int64)
    cov = rng.integers(10, 31, size=n_jobs)
    long_reads = rng.random(n_jobs) < 0.2
    ks = rng.choice(np.array([31, 55]), size=n_jobs)
    out = []
    for j in range(n_jobs):
        out.append(dict(job=j, genome_len=int(G[j]), coverage=int(cov[j]),
                        read_len=10_000 if long_reads[j] else 150,
                        err=0.01 if long_reads[j] else 0.005, k=int(ks[j])))
    return out


def c5_job_reads(spec: dict, seed: int = CONFIG_SEED_BASE + 5, threads: int | None = None):
    """Reads of one served job: a uniform backbone of 90% of its genome plus
    repeat families (length U[1, 6] kbp, 2% divergence) whose copies make up
    the other 10%, sampled at the job's coverage."""
    j = spec["job"]
    G = spec["genome_len"]
    rng = np.random.Generator(np.random.PCG64((seed * 7919 + j) & ((1 << 63) - 1)))
    rep = G // 10
    fams = []
    if rep >= 1000:
        n_f = int(min(5, max(1, rep // 6000)))
        lens = rng.integers(1000, 6001, size=n_f)
        per = rep // n_f
        fams = [(int(l), max(1, int(per // l)), 0.02) for l in lens]
    g = genome(seed * 1000003 + j, max(1000, G - rep), fams)
    rl = spec["read_len"]
    n = max(1, int(g.shape[0]) * spec["coverage"] // rl)
    return reads(g, n, rl, err_rate=spec["err"], seed=seed + 31 * j + 3, threads=threads)


def c5_sample(n_sample: int, n_jobs: int = 10_000, seed: int = CONFIG_SEED_BASE + 5):
    """A seeded subset of the job indices (same distribution)."""
    if n_sample >= n_jobs:
        return list(range(n_jobs))
    rng = np.random.Generator(np.random.PCG64(seed ^ 0xC5))
    return sorted(rng.choice(n_jobs, size=n_sample, replace=False).tolist())
