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
    """Algorithmic HBM bytes of each stage of one call.

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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def h2d_ms(torch, dev, reads: np.ndarray, offs: np.ndarray) -> float:
    """Host-to-device copy of the inputs from pinned host memory (median of 3)."""
    hr = torch.from_numpy(reads).pin_memory()
    ho = torch.from_numpy(offs.view(np.int64)).pin_memory()
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        a = hr.to(dev, non_blocking=True)
        b = ho.to(dev, non_blocking=True)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
        del a, b
    return float(np.median(ts))


def copy_rate(torch, dev, gib: float):
    """Achievable HBM rate: a plain elementwise kernel (bitwise NOT of int64)
    that reads and writes gib GiB each, timed with events on its stream.
    The same kernel calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    if gib <= 0:
        return None
    n = int(gib * (1 << 30)) // 8
    a = torch.empty(n, dtype=torch.int64, device=dev).fill_(0x5A5A)
    b = torch.empty_like(a)
    torch.bitwise_not(a, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        torch.bitwise_not(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * n * 8 / (ms / 1e3) / 1e9, 1)


def traffic_per_launch(kernel: str, config: int, k: int):
    """Measured HBM bytes per launch of `kernel`, from the committed counter
    summary (profiles/traffic.json, written from two rocprofv3 --pmc runs
    scaled by the copy kernel's reading), if it was taken on this workload and
    on the current kernel source; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_2505_04431_amd", "csrc", "kc_kernels.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    ent = rec.get("%s|config%d|k%d" % (kernel, config, k))
    if not ent or ent.get("kernel_source_sha256") != digest:
        return None
    return ent.get("bytes_per_launch")


def batched_leg(n_sample: int, wave_bytes: int, tune: bool, n_small: int = 512) -> dict:
    """Batched workload: read sets of the 4,096-set recipe (genomes log-uniform in
    10 kbp..10 Mbp, 20x of 150 bp reads, 0.5% errors, k in {21, 31}); a seeded
    sample of n_sample sets with the same size distribution. Sets are grouped
    into memory waves of at most wave_bytes; each wave is one recorded-graph
    replay (batched) and, on the same resident inputs, one plain call per set.
    A second figure covers n_small sets of the recipe with genomes of at most
    100 kbp (a third of all sets), where per-call overheads dominate."""
    import torch

    import paper_2505_04431_amd as kc
    import synth
    from paper_2505_04431_amd import tuner
    from concurrent.futures import ThreadPoolExecutor

    dev = torch.device("cuda:0")
    spec = synth.c4_sets()
    tuned = None

    def run_wave(set_ids):
        nonlocal tuned
        t0 = time.time()
        parts, offs, set_reads, set_bytes, ks = [], [np.zeros(1, np.uint64)], [], [], []
        base = 0
        # sets of a wave are laid out by (k, size) so that the plan's classes,
        # which group sets of one k by size, cover contiguous byte ranges
        set_ids = sorted(set_ids, key=lambda i: (spec[i][1], -spec[i][0]))
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            gen = list(ex.map(lambda i: synth.c4_set_reads(i, spec[i][0], threads=1), set_ids))
        for i, (r, o) in zip(set_ids, gen):
            parts.append(r)
            offs.append(o[1:] + np.uint64(base))
            base += r.size
            set_reads.append(o.size - 1)
            set_bytes.append(r.size)
            ks.append(spec[i][1])
        reads = np.concatenate(parts)
        offsets = np.concatenate(offs)
        del parts, gen
        rt = torch.from_numpy(reads).to(dev)
        ot = torch.from_numpy(offsets.view(np.int64)).to(dev)
        del reads
        t_gen = time.time() - t0
        cap = int(sum(set_bytes))
        keys = torch.empty(cap, dtype=torch.int64, device=dev)
        cnts = torch.empty(cap, dtype=torch.int32, device=dev)
        if tuned is None:
            if tune:
                cur = {}

                def run(o):
                    # candidates are tried one after the other: the plan of the
                    # current one is built (and its graph recorded) on its
                    # warm-up call and only its replays are timed; the previous
                    # candidate's plan is freed first
                    key = json.dumps(o, sort_keys=True)
                    if cur.get("key") != key:
                        if "plan" in cur:
                            cur.pop("plan").close()
                        cur["key"] = key
                        cur["plan"] = kc.BatchPlan(set_reads, set_bytes, ks, P=1,
                                                   opts=kc.options(**o))
                    cur["plan"].run_into(rt, ot, keys, cnts, cap)
                    torch.cuda.synchronize()
                tuned = tuner.tune(tuner.class_key("batch", ks, cap), run, reps=2,
                                   use_cache=False)["options"]
                if "plan" in cur:
                    cur.pop("plan").close()
            else:
                tuned = {}
        plan = kc.BatchPlan(set_reads, set_bytes, ks, P=1, opts=kc.options(**tuned))
        plan.run_into(rt, ot, keys, cnts, cap)  # records the graph
        torch.cuda.synchronize()
        t = time.perf_counter()
        n, _ = plan.run_into(rt, ot, keys, cnts, cap)
        torch.cuda.synchronize()
        t_batched = time.perf_counter() - t
        windows = plan.stats()["valid_windows"]
        plan.close()
        # plain: one call per set on the same resident inputs
        st = torch.cuda.current_stream(dev).cuda_stream
        r0 = 0
        bounds = []
        for nr in set_reads:
            bounds.append((r0, r0 + nr))
            r0 += nr
        kc.count_into(rt, ot[bounds[0][0]:bounds[0][1] + 1], ks[0], 1, keys, cnts, cap, None, st)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for (a, b), k in zip(bounds, ks):
            kc.count_into(rt, ot[a:b + 1], k, 1, keys, cnts, cap, None, st)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t
        del rt, ot, keys, cnts
        torch.cuda.empty_cache()
        return dict(windows=windows, bytes=cap, pairs=n, t_batched=t_batched, t_plain=t_plain,
                    t_gen=t_gen)

    idx = synth.c4_sample(n_sample, len(spec))
    sizes = [max(1, spec[i][0] * 20 // 150) * 150 for i in idx]
    groups = synth.waves(sizes, wave_bytes)
    tot = dict(windows=0, bytes=0, t_batched=0.0, t_plain=0.0, t_gen=0.0, pairs=0)
    for gi, grp in enumerate(groups):
        r = run_wave([idx[j] for j in grp])
        for key in tot:
            tot[key] += r[key]
        print("bench: batched wave %d/%d: %d sets, %.2f GB" % (gi + 1, len(groups), len(grp),
                                                              r["bytes"] / 1e9), file=sys.stderr,
              flush=True)
    small = None
    if n_small > 0:
        pool = [i for i, (g, _) in enumerate(spec) if g <= 100_000]
        rng = np.random.Generator(np.random.PCG64(0x5EA11))
        pick = sorted(rng.choice(len(pool), size=min(n_small, len(pool)), replace=False).tolist())
        r = run_wave([pool[j] for j in pick])
        small = {"sets": len(pick), "of_sets_up_to_100kbp": len(pool), "bytes": r["bytes"],
                 "valid_windows": r["windows"],
                 "value": round(r["windows"] / r["t_batched"], 1),
                 "plain_per_set_value": round(r["windows"] / r["t_plain"], 1),
                 "speedup_vs_plain_launches": round(r["t_plain"] / r["t_batched"], 3),
                 "ms_batched": round(r["t_batched"] * 1e3, 3),
                 "ms_plain": round(r["t_plain"] * 1e3, 3)}
    return {
        "workload": "c4_batched_4096_sets_sample", "sets": len(idx), "of_sets": len(spec),
        "waves": len(groups), "wave_bytes": wave_bytes, "bytes": tot["bytes"],
        "valid_windows": tot["windows"], "pairs": tot["pairs"],
        "value": round(tot["windows"] / tot["t_batched"], 1), "unit": "k-mers/s",
        "plain_per_set_value": round(tot["windows"] / tot["t_plain"], 1),
        "speedup_vs_plain_launches": round(tot["t_plain"] / tot["t_batched"], 3),
        "ms_batched": round(tot["t_batched"] * 1e3, 3), "ms_plain": round(tot["t_plain"] * 1e3, 3),
        "tuned_options": tuned,
        "small_sets": small,
        "note": "seeded sample of the 4,096 sets (same size distribution); inputs resident; "
                "one graph replay per wave vs one plain call per set; small_sets: sets with "
                "genomes up to 100 kbp, one wave",
    }


def served_leg(n_jobs: int, budget_gib: float, workers: int, load: float) -> dict:
    """Served workload: a seeded sample of n_jobs of the 10,000-job recipe
    (genomes log-uniform 50 kbp..50 Mbp with 10% repeats, coverage 10-30x,
    80% 150 bp reads at 0.5% errors, 20% 10 kbp reads at 1%, k in {31, 55}).
    Inputs are resident before timing. A calibration pass submits every job
    at once (capacity = jobs / busy time); the timed pass submits them with
    Poisson arrivals at load x capacity and reports throughput and latency."""
    import random
    import threading

    import torch

    import paper_2505_04431_amd as kc
    import synth
    from concurrent.futures import ThreadPoolExecutor

    dev = torch.device("cuda:0")
    specs = synth.c5_jobs()
    idx = synth.c5_sample(n_jobs, len(specs))
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        gen = list(ex.map(lambda j: synth.c5_job_reads(specs[j], threads=1), idx))
    inputs = []
    for (r, o), j in zip(gen, idx):
        inputs.append((torch.from_numpy(r).to(dev), torch.from_numpy(o.view(np.int64)).to(dev),
                       specs[j]["k"]))
    n_bytes = sum(int(r.size) for r, _ in gen)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    budget = int(budget_gib * (1 << 30))
    free0, total0 = torch.cuda.mem_get_info(dev)
    srv = kc.Server(budget, workers)

    def run_pass(arrivals):
        ids = [None] * len(inputs)
        start = time.perf_counter()

        def submitter():
            for i, (rt, ot, k) in enumerate(inputs):
                delay = start + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                ids[i] = srv.submit(rt, ot, k, P=64)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for j in ids:
            assert srv.wait(j) == "done", srv.info(j)
        infos = [srv.info(j) for j in ids]
        for j in ids:
            srv.release(j)
        return infos

    def busy_s(infos):
        return (max(i["t_end_ms"] for i in infos) - min(i["t_start_ms"] for i in infos)) / 1e3

    # a warm-up pass grows every worker's scratch arena (device memory mapped
    # for the first time), then the calibration pass measures capacity
    cold = busy_s(run_pass([0.0] * len(inputs)))
    cal_ms = [busy_s(run_pass([0.0] * len(inputs))) * 1e3 for _ in range(2)]
    capacity = len(inputs) / (min(cal_ms) / 1e3)
    def pct(v, q):
        return round(v[min(len(v) - 1, max(0, int(np.ceil(q * len(v))) - 1))], 3)

    def poisson_pass(ld):
        rng = random.Random(0x5E7)
        arr, t = [], 0.0
        for _ in inputs:
            arr.append(t)
            t += rng.expovariate(ld * capacity)
        g0 = srv.stats()["arena_growths"]
        infos = run_pass(arr)
        growths.append(srv.stats()["arena_growths"] - g0)
        slow.extend({"load": ld, "k": i["k"], "valid_windows": i["valid_windows"],
                     "worker": i["worker"], "wait_ms": round(i["t_start_ms"] - i["t_submit_ms"], 3),
                     "run_ms": round(i["t_end_ms"] - i["t_start_ms"], 3)}
                    for i in sorted(infos, key=lambda i: i["t_start_ms"] - i["t_end_ms"])[:2])
        lat = sorted(i["t_end_ms"] - i["t_submit_ms"] for i in infos)
        wait = sorted(i["t_start_ms"] - i["t_submit_ms"] for i in infos)
        span = (max(i["t_end_ms"] for i in infos) - min(i["t_submit_ms"] for i in infos)) / 1e3
        W = sum(i["valid_windows"] for i in infos)
        return infos, lat, wait, span, W

    slow = []  # the two longest-running jobs of each pass
    growths = []  # arena growths during each Poisson pass
    sweep = []
    for ld in (0.5, 0.9):  # the other arrival rates, beside the headline one
        _, lat_s, _, span_s, W_s = poisson_pass(ld)
        sweep.append({"load": ld, "value": round(W_s / span_s, 1), "arena_growths": growths[-1],
                      "latency_p50_ms": pct(lat_s, 0.5), "latency_p99_ms": pct(lat_s, 0.99)})
    rate = load * capacity
    infos, lat, wait, span, W = poisson_pass(load)
    st = srv.stats()
    srv.close()
    # the host arrays the inputs were copied from outlive the timed passes:
    # freeing GBs of host memory holds the interpreter for tens of ms, which
    # would delay the submitting thread's arrivals
    del gen

    return {
        "workload": "c5_served_10000_jobs_sample", "jobs": len(inputs), "of_jobs": len(specs),
        "bytes": n_bytes, "valid_windows": W, "budget_gib": budget_gib, "workers": workers,
        "value": round(W / span, 1), "unit": "k-mers/s",
        "jobs_per_s": round(len(inputs) / span, 3),
        "capacity_jobs_per_s": round(capacity, 3), "arrival_rate_jobs_per_s": round(rate, 3),
        "cold_pass_ms": round(cold * 1e3, 1), "calibration_ms": [round(x, 1) for x in cal_ms],
        "arena_growths": st["arena_growths"], "scratch_releases": st["scratch_releases"],
        "arena_growths_in_pass": growths[-1],
        "load": load, "latency_p50_ms": pct(lat, 0.5), "latency_p99_ms": pct(lat, 0.99),
        "wait_p50_ms": pct(wait, 0.5), "wait_p99_ms": pct(wait, 0.99),
        "peak_bytes": st["bytes_peak"], "estimate_misses": st["estimate_misses"],
        "gen_s": round(t_gen, 1), "load_sweep": sweep, "longest_jobs": slow,
        "device_free_gb_at_start": round(free0 / 1e9, 1),
        "device_total_gb": round(total0 / 1e9, 1),
        "note": "seeded sample of the 10,000 jobs (same distribution); inputs resident; Poisson "
                "arrivals at load x capacity (all jobs at once, the faster of two calibration "
                "passes after a warm-up pass; cold_pass_ms: the warm-up's busy time, arenas grown "
                "from nothing); latency = completion - submission",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--batched-sets", type=int, default=256,
                    help="sets of the batched workload to run (0: skip the batched leg)")
    ap.add_argument("--wave-gb", type=float, default=2.0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--served-jobs", type=int, default=32,
                    help="jobs of the served workload to run (0: skip the served leg)")
    ap.add_argument("--served-budget-gib", type=float, default=192.0)
    ap.add_argument("--served-workers", type=int, default=4)
    ap.add_argument("--served-load", type=float, default=0.7)
    ap.add_argument("--sort-steps", type=int, default=5,
                    help="calls of the sort-based leaf count to time (0: skip)")
    ap.add_argument("--fastq-steps", type=int, default=5,
                    help="calls of the FASTQ parser on the workload's reads as FASTQ text "
                         "(0: skip)")
    ap.add_argument("--long-k", type=int, default=100,
                    help="k of the long-key leg (65..128: four-word keys, sort-based leaves)")
    ap.add_argument("--long-k-steps", type=int, default=3,
                    help="calls of the long-key leg to time (0: skip)")
    ap.add_argument("--stream-pieces", type=int, default=4,
                    help="pieces of the streamed leg: the reads counted from host memory in "
                         "pieces whose results are merged (0: skip)")
    ap.add_argument("--copy-gib", type=float, default=1.0,
                    help="size of the plain copy kernel timed for the achievable HBM rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this path counts on one GPU only; --gpus %d is not supported "
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
    step_ms = []
    t_start = time.perf_counter()
    n_out = 0
    for _ in range(args.steps):
        # each call returns with its output complete (it synchronises its stream)
        t1 = time.perf_counter()
        n_out = kc.count_into(rt, ot, k, P, keys, cnts, cap, opts, stream.cuda_stream)
        step_ms.append((time.perf_counter() - t1) * 1e3)
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
                    "k_leaf_countw<u128, 512, 2048, 4>"}
    copy_gbs = copy_rate(torch, dev, args.copy_gib)
    ceil = kc.kc.measure_ceilings(4 << 30, stream.cuda_stream)
    t_h2d = h2d_ms(torch, dev, reads, offs)
    kname = kernel_names.get(dom, dom)
    traffic = traffic_per_launch(kname, args.config, k)
    roofline = {"bound": "hbm", "kernel": kname, "stage": dom,
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_unit": "bytes per launch",
                "traffic_gbs": round(traffic / (avg[dom] / 1e3) / 1e9, 1) if traffic else None,
                "copy_gbs": copy_gbs,
                "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
                "leaf_records_per_s": round(st["large_records"] / (avg[dom] / 1e3), 1)
                if dom == "leaf_large" else None,
                "ceilings": {n: (round(v, 2) if isinstance(v, float) else v)
                             for n, v in ceil.items()},
                "leaf_inserts_frac_of_lds_ceiling": round(
                    st["large_records"] / (avg[dom] / 1e3) / (ceil["lds_insert_gops"] * 1e9), 4)
                if dom == "leaf_large" else None,
                "stage_ms": {n: round(v, 4) for n, v in avg.items()},
                "stage_gbs": {n: round(sb[n] / (avg[n] / 1e3) / 1e9, 1) for n in avg if n in sb}}

    # the paper's own counting step (sort + run-length accumulate of each
    # owner's records) on the same partitions, for comparison
    sort_mode = None
    if args.sort_steps > 0:
        o1 = kc.options(timing=1, mode=1)
        kc.count_into(rt, ot, k, P, keys, cnts, cap, o1, stream.cuda_stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        leaf1 = 0.0
        for _ in range(args.sort_steps):
            kc.count_into(rt, ot, k, P, keys, cnts, cap, o1, stream.cuda_stream)
            leaf1 += kc.last_stats()["ms_stage"]["leaf_large"]
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - t1) * 1e3 / args.sort_steps
        sort_mode = {"value": round(W / (ms1 / 1e3), 1), "unit": "k-mers/s",
                     "ms_per_step": round(ms1, 4),
                     "leaf_ms": round(leaf1 / args.sort_steps, 4),
                     "note": "kc_options.mode = 1: each leaf's records sorted in LDS and "
                             "run-length accumulated instead of counted in a hash table"}

    # the same reads as FASTQ text on the device: parse, then count the parsed reads
    fastq = None
    if args.fastq_steps > 0:
        text = synth.to_fastq(reads, offs, seed=1)
        tt = torch.frombuffer(bytearray(text), dtype=torch.uint8).to(dev)
        del text
        pr, po, _ = kc.parse_fastx(tt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.fastq_steps):
            pr, po, _ = kc.parse_fastx(tt)
        torch.cuda.synchronize()
        ms_p = (time.perf_counter() - t1) * 1e3 / args.fastq_steps
        ok = pr.numel() == reads.size and po.numel() == offs.size
        t1 = time.perf_counter()
        for _ in range(args.fastq_steps):
            pr, po, _ = kc.parse_fastx(tt)
            kc.count_into(pr, po, k, P, keys, cnts, cap, None, stream.cuda_stream)
        torch.cuda.synchronize()
        ms_pc = (time.perf_counter() - t1) * 1e3 / args.fastq_steps
        fastq = {"text_bytes": tt.numel(), "records": po.numel() - 1, "parsed_whole": ok,
                 "parse_ms": round(ms_p, 4), "parse_gbs": round(tt.numel() / (ms_p / 1e3) / 1e9, 1),
                 "parse_and_count_ms": round(ms_pc, 4),
                 "from_text_value": round(W / (ms_pc / 1e3), 1), "unit": "k-mers/s",
                 "note": "kc_parse_fastx on the FASTQ text of the same reads (random "
                         "qualities), then kc_count on its output"}
        del tt, pr, po

    # the reads in pinned host memory, counted in pieces whose copies overlap
    # the counts, each piece's result merged on the device
    streamed = None
    if args.stream_pieces > 0:
        chunk = (reads.size + args.stream_pieces - 1) // args.stream_pieces
        host_pinned = torch.from_numpy(reads).pin_memory()
        kc.count_chunked(host_pinned, offs, k, P, chunk_bytes=chunk)
        torch.cuda.synchronize()
        reps = 3
        t1 = time.perf_counter()
        for _ in range(reps):
            sk_, sc_ = kc.count_chunked(host_pinned, offs, k, P, chunk_bytes=chunk)
        torch.cuda.synchronize()
        ms_s = (time.perf_counter() - t1) * 1e3 / reps
        streamed = {"pieces": args.stream_pieces, "ms_per_step": round(ms_s, 4),
                    "value": round(W / (ms_s / 1e3), 1), "unit": "k-mers/s",
                    "same_distinct": int(sc_.numel()) == n_out,
                    "note": "reads in pinned host memory counted in pieces (kc_count per "
                            "piece, kc_merge_counts into the running result); the next "
                            "piece's host-to-device copy overlaps the count; every copy is "
                            "inside the time"}
        del sk_, sc_, host_pinned

    # the legs above leave this thread's scratch arena sized for their largest
    # call (32-byte records for the long keys); the batched and served legs
    # start from released device memory
    kc.lib().kc_release_scratch()
    torch.cuda.empty_cache()

    batched = None
    if args.batched_sets > 0:
        batched = batched_leg(args.batched_sets, int(args.wave_gb * 1e9), not args.no_tune)

    served = None
    if args.served_jobs > 0:
        kc.lib().kc_release_scratch()
        torch.cuda.empty_cache()
        served = served_leg(args.served_jobs, args.served_budget_gib, args.served_workers,
                            args.served_load)

    # keys of more than 64 bases on the same reads (last: its 32-byte records
    # size this thread's scratch arena far above the other legs')
    long_k = None
    if args.long_k_steps > 0:
        kl = args.long_k
        cap_l = kc.max_outputs(offs, kl)
        keys_l = torch.empty((max(cap_l, 1), 4), dtype=torch.int64, device=dev)
        cnts_l = torch.empty(max(cap_l, 1), dtype=torch.int32, device=dev)
        ol = kc.options(timing=1)
        kc.count_into(rt, ot, kl, P, keys_l, cnts_l, max(cap_l, 1), ol, stream.cuda_stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        leaf_l = 0.0
        for _ in range(args.long_k_steps):
            n_l = kc.count_into(rt, ot, kl, P, keys_l, cnts_l, max(cap_l, 1), ol,
                                stream.cuda_stream)
            leaf_l += kc.last_stats()["ms_stage"]["leaf_large"]
        torch.cuda.synchronize()
        ms_l = (time.perf_counter() - t1) * 1e3 / args.long_k_steps
        st_l = kc.last_stats()
        long_k = {"k": kl, "value": round(st_l["valid_windows"] / (ms_l / 1e3), 1),
                  "unit": "k-mers/s", "ms_per_step": round(ms_l, 4),
                  "leaf_ms": round(leaf_l / args.long_k_steps, 4),
                  "valid_windows": st_l["valid_windows"], "distinct": n_l,
                  "note": "256-bit keys (four words); LDS tables whose slots are claimed "
                          "through their 64-bit count word"}
        del keys_l, cnts_l

    # the CPU oracle runs after every GPU leg, so that its host allocations
    # (several GB, 16 threads) do not overlap the served leg's host-side work
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
        # one thread on a sixteenth of the reads
        n_1 = max(1, n_s // 16)
        r_1, o_1 = reads[:int(offs[n_1])], offs[:n_1 + 1]
        w_1 = oracle.valid_windows(r_1, o_1, k)
        tc = time.perf_counter()
        oracle.count(r_1, o_1, k, threads=1)
        dt1 = time.perf_counter() - tc
        cpu = {"value": round(w_s / dt, 1), "unit": "k-mers/s", "cores": threads, "kind": "oracle",
               "sample": "first %d of %d reads (%d valid windows), sort-based oracle, %d threads"
                         % (n_s, len(offs) - 1, w_s, threads),
               "one_thread_value": round(w_1 / dt1, 1),
               "one_thread_sample": "first %d reads (%d valid windows)" % (n_1, w_1),
               "cpu_model": cpu_model()}

    line = {
        "metric": "canonical k-mers counted/sec on 1 MI355X + % HBM roofline; batched vs plain",
        "value": round(value, 1), "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "ms_median": round(float(np.median(step_ms)), 4), "ms_best": round(min(step_ms), 4),
        "h2d_ms": round(t_h2d, 4),
        "end_to_end_value": round(W / ((ms_step + t_h2d) / 1e3), 1),
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if k <= 32 else "u128",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "k": k, "P": P, "reads": len(offs) - 1,
                   "read_len": 150, "valid_windows": W, "distinct": n_out, "mode": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "sort_mode": sort_mode,
        "fastq": fastq,
        "streamed": streamed,
        "long_k": long_k,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
