"""Benchmark: canonical k-mers counted per second on one MI355X.

Workload (one step = one full pass of the counting path): 5,000,000 bp uniform
genome plus 5 repeat families (1-6 kbp, 40 copies each at 2% divergence),
1,000,000 reads of 150 bp on random strands with 1% substitutions and 0.01% N,
k = 31, P = 64 owner partitions. Inputs are generated on the host, copied to
HBM before the timed region, and stay resident.

value = valid windows (canonical k-mers counted) / seconds per step.
Prints one JSON line. With --gpus N > 1 it exits: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def stage_bytes(st: dict, k: int) -> dict:
    """Algorithmic HBM bytes of each stage of one call (the bytes model in the design doc).

    N bases, W valid windows, D distinct keys, K key bytes (8 for k <= 32, else 16).
    Records are written once by the owner scatter, read by the split histogram,
    read and written by the split scatter, read by the leaf count, which writes
    (key, count) pairs that the concat reads and writes to the output.
    """
    N = st["n_bases"]
    W = st["valid_windows"]
    D = st["distinct"]
    K = 16 if k > 32 else 8
    packed = N / 4 + N / 8 + N / 8          # 2-bit bases + invalid mask + read-end mask
    return {
        "pack": N + packed,                  # read ASCII, write packed + masks
        "window_hist": packed,               # read packed + masks
        "owner_scatter": packed + K * W,     # read packed, write one record per window
        "split_hist": K * W,                 # read records
        "split_scatter": 2 * K * W,          # read + write records
        "leaf_large": K * st["large_records"] + (K + 4) * st["large_distinct"],
        "leaf_small": K * (W - st["large_records"]) + (K + 4) * (D - st["large_distinct"]),
        "concat": 2 * (K + 4) * D,           # read pairs, write output
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--k", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build counts on one GPU only; --gpus %d is not supported "
              "(run with --gpus 1)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_2505_04431_amd as kc
    import synth

    t0 = time.time()
    cfg = synth.make_config(args.config)
    k = args.k or cfg["ks"][0]
    P = cfg["P"]
    reads, offs = cfg["reads"], cfg["offsets"]
    dev = torch.device("cuda:0")
    rt = torch.from_numpy(reads).to(dev)
    ot = torch.from_numpy(offs.view(np.int64)).to(dev)
    cap = kc.max_outputs(offs, k)
    words = 2 if k > 32 else 1
    keys = torch.empty((cap, words) if words == 2 else (cap,), dtype=torch.int64, device=dev)
    cnts = torch.empty(cap, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    opts = kc.options(timing=1)
    torch.cuda.synchronize()
    print("bench: inputs ready in %.1fs (%d reads, %d bytes)" % (time.time() - t0, len(offs) - 1,
                                                                  reads.size),
          file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        kc.count_into(rt, ot, k, P, keys, cnts, cap, opts, stream.cuda_stream)
    torch.cuda.synchronize()
    stage_ms: dict = {}
    t_start = time.perf_counter()
    n_out = 0
    for _ in range(args.steps):
        n_out = kc.count_into(rt, ot, k, P, keys, cnts, cap, opts, stream.cuda_stream)
        st = kc.last_stats()
        for name, ms in st["ms_stage"].items():
            stage_ms[name] = stage_ms.get(name, 0.0) + ms
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = elapsed * 1e3 / args.steps
    W = st["valid_windows"]
    value = W / (ms_step / 1e3)

    avg = {n: v / args.steps for n, v in stage_ms.items() if v > 0}
    sb = stage_bytes(st, k)
    dom = max((n for n in avg if n in sb), key=lambda n: avg[n])
    achieved = sb[dom] / (avg[dom] / 1e3) / 1e9
    kernel_names = {"leaf_large": "k_leaf_count64<512, 4096, 4>" if k <= 32 else
                    "k_leaf_count128<512, 2048, 4>"}
    roofline = {"bound": "hbm", "kernel": kernel_names.get(dom, dom), "stage": dom,
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None,
                "stage_ms": {n: round(v, 4) for n, v in avg.items()},
                "stage_gbs": {n: round(sb[n] / (avg[n] / 1e3) / 1e9, 1) for n in avg if n in sb}}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        # bounded sample: the whole workload is about 10 s of oracle work on 16 threads
        n_s = len(offs) - 1
        r_s, o_s = reads[:int(offs[n_s])], offs[:n_s + 1]
        w_s = oracle.valid_windows(r_s, o_s, k)
        tc = time.perf_counter()
        oracle.count(r_s, o_s, k, threads=threads)
        dt = time.perf_counter() - tc
        cpu = {"value": round(w_s / dt, 1), "unit": "k-mers/s", "cores": threads, "kind": "oracle",
               "sample": "first %d of %d reads (%d valid windows), sort-based oracle, %d threads"
                         % (n_s, len(offs) - 1, w_s, threads)}

    line = {
        "metric": "canonical k-mers counted/sec on 1 MI355X + % HBM roofline; batched vs plain",
        "value": round(value, 1), "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if k <= 32 else "u128",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "k": k, "P": P, "reads": len(offs) - 1,
                   "read_len": 150, "valid_windows": W, "distinct": n_out, "mode": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
