"""Benchmark: canonical k-mers counted per second on one MI355X.

Headline workload (one step = one full pass of the counting path, kc_count):
a 200 Mbp genome (110 Mbp of uniform ACGT plus 90 Mbp from 50 repeat families
with Zipf(1.2) copy numbers capped at 10^4, 2-5% divergence), 40,000,000 reads
of 150 bp at 30x on random strands with 0.5% substitutions, k = 31, P = 256
owner partitions; k = 21 on the same reads is the second figure. Inputs are
generated on the host, copied to HBM before the timed region, and stay
resident. Secondary legs: the 1,000,000-read workload (5 Mbp + repeats, 1%
errors, 0.01% N, k = 31, P = 64) with the sort-based leaves, FASTQ parsing,
counting from host memory in pieces and 256-bit keys; the batched workload
(all 4,096 read sets, memory waves planned by the library) against one plain
call per set; the served workload (500 jobs of the 10,000-job recipe, Poisson
arrivals, p50/p99 latency); the CPU oracle on a sample of the headline reads.

value = valid windows (canonical k-mers counted) / seconds per step.
Prints one JSON line. With --gpus N > 1 it exits: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "canonical k-mers counted/sec on 1 MI355X + % HBM roofline; batched vs plain"


def stage_bytes(st: dict, k: int) -> dict:
    """Algorithmic HBM bytes of each stage of one call.

    N bases, W valid windows, D distinct keys, K key bytes (8 for k <= 32,
    16 for k <= 64). Records are written once by the owner scatter, read by
    the split histogram, read and written by the split scatter, read by the
    leaf count, which writes (key, count) pairs that the concat reads and
    writes to the output. The block-wide leaf kernel's launch reads its
    records (large_records) and writes its pairs (large_distinct); the second
    count of the leaves whose table overflowed likewise (second_records,
    second_distinct).
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
        "leaf_second": K * st["second_records"] + (K + 4) * st["second_distinct"],
        "concat": 2 * (K + 4) * D,           # read pairs, write output
    }


KERNEL_NAMES = {  # rocprofv3 names of the kernel behind each single-kernel stage
    ("leaf_large", 1): "k_leaf_count64<512, 4096, 4, false, false>",
    ("leaf_large", 2): "k_leaf_countw<unsigned __int128, 512, 2048, 4, true, false>",
    ("leaf_second", 1): "k_leaf_count64<1024, 8192, 4, true, false>",
    ("split_scatter", 1): "k_split_scatter<unsigned long, 1024, 16>",
    ("owner_scatter", 1): "k_window_scatter64<unsigned long, unsigned long, 8, 1024, false>",
    ("window_hist", 1): "k_window_hist<unsigned long, unsigned long, 8, 256, false>",
    ("split_hist", 1): "k_split_hist<unsigned long, 256>",
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


def host_cores() -> tuple[int, dict]:
    """Cores this process may use: its CPU affinity, capped by a cgroup CPU
    quota when one is set. Returns (cores, details)."""
    aff = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, p = f.read().split()[:2]
            if q != "max":
                quota = int(q) / int(p)
    except (OSError, ValueError):
        pass
    cores = aff if quota is None else max(1, min(aff, int(quota)))
    return cores, {"affinity": aff, "cgroup_quota": quota, "cpu_count": os.cpu_count()}


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
    del hr, ho
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


def traffic_per_launch(kernel: str, workload: str, k: int):
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
    ent = rec.get("%s|%s|k%d" % (kernel, workload, k))
    if not ent or ent.get("kernel_source_sha256") != digest:
        return None
    return ent.get("bytes_per_launch")


def timed_steps(kc, torch, rt, ot, k, P, keys, cnts, cap, steps, warmup, stream):
    """warmup untimed calls, then `steps` timed ones (each returns with its
    output complete); per-stage device times from the events the library
    records on the call's stream."""
    opts = kc.options(timing=1)
    for _ in range(warmup):
        kc.count_into(rt, ot, k, P, keys, cnts, cap, opts, stream)
    torch.cuda.synchronize()
    stage_ms: dict = {}
    step_ms = []
    n_out = 0
    st = None
    t_start = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        n_out = kc.count_into(rt, ot, k, P, keys, cnts, cap, opts, stream)
        step_ms.append((time.perf_counter() - t1) * 1e3)
        st = kc.last_stats()
        for name, ms in st["ms_stage"].items():
            stage_ms[name] = stage_ms.get(name, 0.0) + ms
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    avg = {n: v / steps for n, v in stage_ms.items() if v > 0}
    return dict(ms_step=elapsed * 1e3 / steps, step_ms=step_ms, avg=avg, st=st, n_out=n_out)


def roofline_of(run: dict, k: int, workload: str, copy_gbs, ceil=None) -> dict:
    """Roofline of the dominant single-kernel stage of a timed run."""
    st, avg = run["st"], run["avg"]
    sb = stage_bytes(st, k)
    words = 1 if k <= 32 else 2
    dom = max((n for n in avg if n in sb), key=lambda n: avg[n])
    achieved = sb[dom] / (avg[dom] / 1e3) / 1e9
    kname = KERNEL_NAMES.get((dom, words), dom)
    traffic = traffic_per_launch(kname, workload, k)
    out = {"bound": "hbm", "kernel": kname, "stage": dom, "achieved": round(achieved, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": traffic, "traffic_unit": "bytes per launch",
           "algorithmic_bytes": round(sb[dom]), "kernel_ms": round(avg[dom], 4),
           "traffic_gbs": round(traffic / (avg[dom] / 1e3) / 1e9, 1) if traffic else None,
           "copy_gbs": copy_gbs,
           "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
           "stage_ms": {n: round(v, 4) for n, v in avg.items()},
           "stage_gbs": {n: round(sb[n] / (avg[n] / 1e3) / 1e9, 1) for n in avg if n in sb}}
    if dom == "leaf_large":
        rate = st["large_records"] / (avg[dom] / 1e3)
        out["leaf_records_per_s"] = round(rate, 1)
        if ceil:
            out["leaf_inserts_frac_of_lds_ceiling"] = round(rate / (ceil["lds_insert_gops"] * 1e9), 4)
    return out


def batched_leg(n_sets: int, budget_gib: float, tune: bool) -> dict:
    """Batched workload: the read sets of the 4,096-set recipe (genomes
    log-uniform in 10 kbp..10 Mbp, 20x of 150 bp reads, 0.5% errors, k in
    {21, 31}), the first n_sets of them in (k, size) order. The library plans
    memory waves under a device budget; each wave's reads are generated on
    the host while the previous wave counts, copied to the device, counted by
    its recorded graph (first run: record + count; timed: the replay), and
    counted again by one plain call per set on the same resident inputs."""
    import torch

    import paper_2505_04431_amd as kc
    import synth
    from concurrent.futures import ThreadPoolExecutor
    from paper_2505_04431_amd import tuner

    dev = torch.device("cuda:0")
    spec = synth.c4_sets()
    ids = sorted(range(len(spec)), key=lambda i: (spec[i][1], -spec[i][0]))[:n_sets]
    n_reads = [max(1, spec[i][0] * 20 // 150) for i in ids]
    set_bytes = [n * 150 for n in n_reads]
    ks = [spec[i][1] for i in ids]
    budget = int(budget_gib * (1 << 30))
    cores, _ = host_cores()
    pool = ThreadPoolExecutor(max_workers=max(1, min(16, cores)))

    def gen_wave(w):
        a, b = w["first_set"], w["first_set"] + w["n_sets"]
        parts = list(pool.map(lambda i: synth.c4_set_reads(i, spec[i][0], threads=1), ids[a:b]))
        reads = np.concatenate([r for r, _ in parts])
        offs = [np.zeros(1, np.uint64)]
        base = 0
        for r, o in parts:
            offs.append(o[1:] + np.uint64(base))
            base += r.size
        return reads, np.concatenate(offs)

    def tune_group(lo, hi):
        """Options timed on the first wave of the sets [lo, hi) (one k)."""
        plan = kc.BatchPlan(n_reads[lo:hi], set_bytes[lo:hi], ks[lo:hi], P=1, hbm_budget=budget)
        w0 = plan.waves[0]
        plan.close()
        a, b = lo + w0["first_set"], lo + w0["first_set"] + w0["n_sets"]
        r0, o0 = gen_wave({"first_set": a, "n_sets": b - a})
        rt = torch.from_numpy(r0).to(dev)
        ot = torch.from_numpy(o0.view(np.int64)).to(dev)
        cap = max(1, r0.size // 2)
        keys = torch.empty(cap, dtype=torch.int64, device=dev)
        cnts = torch.empty(cap, dtype=torch.int32, device=dev)
        cur = {}

        def run(o):
            key = json.dumps(o, sort_keys=True)
            if cur.get("key") != key:
                if "plan" in cur:
                    cur.pop("plan").close()
                cur["key"] = key
                cur["plan"] = kc.BatchPlan(n_reads[a:b], set_bytes[a:b], ks[a:b], P=1,
                                           opts=kc.options(**o))
            cur["plan"].run_into(rt, ot, keys, cnts, cap)
            torch.cuda.synchronize()
        cands = [{}, {"split_tile": 8}, {"scatter_tile": 16}, {"leaf_target": 3072},
                 {"leaf_target": 8192}, {"table_slots_log2": 11}]
        info = tuner.tune(tuner.class_key("batch", ks[a:b], r0.size), run, candidates=cands,
                          reps=2, use_cache=False)
        if "plan" in cur:
            cur.pop("plan").close()
        del rt, ot, keys, cnts
        return info

    # one plan per k (the sets are in k order), tuned on its own first wave:
    # the best leaf size differs between one-word keys and the two-word keys
    # of k = 31 classes
    groups = []
    lo = 0
    while lo < len(ks):
        hi = lo
        while hi < len(ks) and ks[hi] == ks[lo]:
            hi += 1
        groups.append((lo, hi))
        lo = hi
    tot = dict(windows=0, bytes=0, pairs=0, t_first=0.0, t_batched=0.0, t_plain=0.0, t_gen=0.0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    t_leg = time.time()
    tuned_by_k, tuning_by_k = {}, {}
    n_waves, max_wave_bytes = 0, 0
    for lo, hi in groups:
        info = tune_group(lo, hi) if tune else None
        tuned = info["options"] if info else {}
        tuned_by_k[str(ks[lo])] = tuned
        tuning_by_k[str(ks[lo])] = info["timings"] if info else None
        plan = kc.BatchPlan(n_reads[lo:hi], set_bytes[lo:hi], ks[lo:hi], P=1,
                            hbm_budget=budget, opts=kc.options(**tuned))
        waves = [dict(w, first_set=w["first_set"] + lo) for w in plan.waves]
        n_waves += len(waves)
        max_wave_bytes = max([max_wave_bytes] + [w["device_bytes"] for w in waves])
        gen_pool = ThreadPoolExecutor(max_workers=1)
        nxt = gen_pool.submit(gen_wave, waves[0]) if waves else None
        for wi, w in enumerate(waves):
            t0 = time.time()
            reads, offs = nxt.result()
            tot["t_gen"] += time.time() - t0
            if wi + 1 < len(waves):
                nxt = gen_pool.submit(gen_wave, waves[wi + 1])  # overlaps this wave's counting
            rt = torch.from_numpy(reads).to(dev)
            ot = torch.from_numpy(offs.view(np.int64)).to(dev)
            cap = max(1, reads.size // 2)
            keys = torch.empty(cap, dtype=torch.int64, device=dev)
            cnts = torch.empty(cap, dtype=torch.int32, device=dev)
            torch.cuda.synchronize()
            t = time.perf_counter()
            n, _ = plan.run_wave_into(wi, rt, ot, keys, cnts, cap, stream)  # records the graph
            torch.cuda.synchronize()
            tot["t_first"] += time.perf_counter() - t
            t = time.perf_counter()
            n, set_off = plan.run_wave_into(wi, rt, ot, keys, cnts, cap, stream)
            torch.cuda.synchronize()
            tot["t_batched"] += time.perf_counter() - t
            windows = plan.stats()["valid_windows"]
            # plain: one call per set on the same resident inputs
            r0 = 0
            bounds = []
            for s in range(w["first_set"], w["first_set"] + w["n_sets"]):
                bounds.append((r0, r0 + n_reads[s], ks[s]))
                r0 += n_reads[s]
            t = time.perf_counter()
            for a, b, k in bounds:
                kc.count_into(rt, ot[a:b + 1], k, 1, keys, cnts, cap, None, stream)
            torch.cuda.synchronize()
            tot["t_plain"] += time.perf_counter() - t
            tot["windows"] += windows
            tot["bytes"] += reads.size
            tot["pairs"] += n
            print("bench: batched k=%d wave %d/%d: %d sets, %.2f GB, %.1f ms batched, %.1f ms plain"
                  % (ks[lo], wi + 1, len(waves), w["n_sets"], reads.size / 1e9,
                     tot["t_batched"] * 1e3, tot["t_plain"] * 1e3), file=sys.stderr, flush=True)
            del rt, ot, keys, cnts, reads, offs
        gen_pool.shutdown()
        plan.close()
    pool.shutdown()
    torch.cuda.empty_cache()
    return {
        "workload": "c4_batched_4096_sets", "sets": len(ids), "of_sets": len(spec),
        "waves": n_waves, "hbm_budget_gib": budget_gib,
        "max_wave_device_bytes": max_wave_bytes,
        "bytes": tot["bytes"], "valid_windows": tot["windows"], "pairs": tot["pairs"],
        "value": round(tot["windows"] / tot["t_batched"], 1), "unit": "k-mers/s",
        "value_with_graph_recording": round(tot["windows"] / tot["t_first"], 1),
        "plain_per_set_value": round(tot["windows"] / tot["t_plain"], 1),
        "speedup_vs_plain_launches": round(tot["t_plain"] / tot["t_batched"], 3),
        "ms_batched": round(tot["t_batched"] * 1e3, 3), "ms_plain": round(tot["t_plain"] * 1e3, 3),
        "ms_first_runs": round(tot["t_first"] * 1e3, 3),
        "host_wait_for_generation_s": round(tot["t_gen"], 1),
        "leg_s": round(time.time() - t_leg, 1),
        "tuned_options": tuned_by_k,
        "tuning": tuning_by_k,
        "note": "every set of the recipe, in (k, size) order; one plan per k, its options tuned "
                "on its first wave; waves planned by kc_batch_plan under the budget; each wave's "
                "inputs generated on the host while the previous wave counts; value: graph "
                "replays; plain: one kc_count per set on the same resident inputs",
    }


def served_leg(n_jobs: int, budget_gib: float, workers: int, load: float) -> dict:
    """Served workload: a seeded sample of n_jobs of the 10,000-job recipe
    (genomes log-uniform 50 kbp..50 Mbp with 10% repeats, coverage 10-30x,
    80% 150 bp reads at 0.5% errors, 20% 10 kbp reads at 1%, k in {31, 55}).
    Inputs are resident before timing. A client thread releases each result as
    soon as its job is done. Each job's distinct-key reservation is the size
    predictor's estimate, from a predictor trained on the other half of the
    jobs (two-fold: no job's hint comes from a model that saw it). A warm-up
    pass and a calibration pass submit every job at once (capacity = jobs /
    busy time); the timed passes submit them with Poisson arrivals at load x
    capacity and report throughput and latency."""
    import random

    import torch

    import paper_2505_04431_amd as kc
    import synth
    from concurrent.futures import ThreadPoolExecutor
    from paper_2505_04431_amd import predictor as pred

    dev = torch.device("cuda:0")
    specs = synth.c5_jobs()
    idx = synth.c5_sample(n_jobs, len(specs))
    t0 = time.time()
    cores, _ = host_cores()
    inputs = []
    with ThreadPoolExecutor(max_workers=max(1, min(16, cores))) as ex:
        for (r, o), j in zip(ex.map(lambda j: synth.c5_job_reads(specs[j], threads=1), idx), idx):
            inputs.append((torch.from_numpy(r).to(dev), torch.from_numpy(o.view(np.int64)).to(dev),
                           specs[j]["k"]))
    n_bytes = sum(int(r.numel()) for r, _, _ in inputs)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    budget = int(budget_gib * (1 << 30))
    free0, total0 = torch.cuda.mem_get_info(dev)
    srv = kc.Server(budget, workers)

    def run_pass(arrivals, hints):
        ids = [None] * len(inputs)
        start = time.perf_counter()
        infos = [None] * len(inputs)

        def submitter():
            for i, (rt, ot, k) in enumerate(inputs):
                delay = start + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                ids[i] = srv.submit(rt, ot, k, P=64, distinct_hint=hints[i])

        th = threading.Thread(target=submitter)
        th.start()
        # the client: every finished job is read and released at once
        left = set(range(len(inputs)))
        while left:
            done_any = False
            for i in list(left):
                if ids[i] is None:
                    continue
                s = srv.poll(ids[i])
                if s in ("done", "failed"):
                    infos[i] = srv.info(ids[i])
                    assert s == "done", infos[i]
                    srv.release(ids[i])
                    left.discard(i)
                    done_any = True
            if not done_any:
                time.sleep(0.0002)
        th.join()
        return infos

    def busy_s(infos):
        return (max(i["t_end_ms"] for i in infos) - min(i["t_start_ms"] for i in infos)) / 1e3

    no_hint = [0] * len(inputs)
    cold_infos = run_pass([0.0] * len(inputs), no_hint)  # grows the workers' arenas
    cold = busy_s(cold_infos)
    # size predictor: features of every job, two-fold training on the true
    # distinct counts of the warm-up pass
    feats = np.stack([pred.job_features(rt, ot, k, P=64)[0] for rt, ot, k in inputs])
    ln_d = np.log(np.maximum(1, np.array([i["distinct"] for i in cold_infos], np.float64)))
    hints = [0] * len(inputs)
    fold = np.arange(len(inputs)) % 2
    for f in (0, 1):
        tr, te = np.flatnonzero(fold != f), np.flatnonzero(fold == f)
        model = pred.SizePredictor()
        model.fit(feats[tr], ln_d[tr], steps=2000)
        for i in te:
            hints[i] = model.hint(feats[i])
        model.close()
    cal_ms = busy_s(run_pass([0.0] * len(inputs), hints)) * 1e3
    capacity = len(inputs) / (cal_ms / 1e3)

    def pct(v, q):
        return round(v[min(len(v) - 1, max(0, int(np.ceil(q * len(v))) - 1))], 3)

    growths = []
    slow = []

    def poisson_pass(ld):
        rng = random.Random(0x5E7)
        arr, t = [], 0.0
        for _ in inputs:
            arr.append(t)
            t += rng.expovariate(ld * capacity)
        g0 = srv.stats()["unplaced"]
        infos = run_pass(arr, hints)
        growths.append(srv.stats()["unplaced"] - g0)
        slow.extend({"load": ld, "k": i["k"], "valid_windows": i["valid_windows"],
                     "worker": i["worker"], "wait_ms": round(i["t_start_ms"] - i["t_submit_ms"], 3),
                     "run_ms": round(i["t_end_ms"] - i["t_start_ms"], 3)}
                    for i in sorted(infos, key=lambda i: i["t_start_ms"] - i["t_end_ms"])[:2])
        lat = sorted(i["t_end_ms"] - i["t_submit_ms"] for i in infos)
        wait = sorted(i["t_start_ms"] - i["t_submit_ms"] for i in infos)
        span = (max(i["t_end_ms"] for i in infos) - min(i["t_submit_ms"] for i in infos)) / 1e3
        W = sum(i["valid_windows"] for i in infos)
        res_est = sum(i["result_estimate_bytes"] for i in infos)
        res_act = sum(i["result_bytes"] for i in infos)
        under = sum(1 for i in infos if i["result_bytes"] > i["result_estimate_bytes"])
        return infos, lat, wait, span, W, res_est, res_act, under

    sweep = []
    for ld in (0.5, 0.9):  # the other arrival rates, beside the headline one
        _, lat_s, _, span_s, W_s, _, _, _ = poisson_pass(ld)
        sweep.append({"load": ld, "value": round(W_s / span_s, 1), "unplaced_waits": growths[-1],
                      "latency_p50_ms": pct(lat_s, 0.5), "latency_p99_ms": pct(lat_s, 0.99)})
    rate = load * capacity
    infos, lat, wait, span, W, res_est, res_act, under = poisson_pass(load)
    st = srv.stats()
    srv.close()
    no_hint_reserved = sum(i["result_estimate_bytes"] for i in cold_infos)
    return {
        "workload": "c5_served_10000_jobs_sample", "jobs": len(inputs), "of_jobs": len(specs),
        "bytes": n_bytes, "valid_windows": W, "budget_gib": budget_gib, "workers": workers,
        "value": round(W / span, 1), "unit": "k-mers/s",
        "jobs_per_s": round(len(inputs) / span, 3),
        "capacity_jobs_per_s": round(capacity, 3), "arrival_rate_jobs_per_s": round(rate, 3),
        "cold_pass_ms": round(cold * 1e3, 1), "calibration_ms": round(cal_ms, 1),
        "slab_bytes": st["slab_bytes"], "unplaced_waits": st["unplaced"],
        "unplaced_waits_in_pass": growths[-1],
        "load": load, "latency_p50_ms": pct(lat, 0.5), "latency_p99_ms": pct(lat, 0.99),
        "wait_p50_ms": pct(wait, 0.5), "wait_p99_ms": pct(wait, 0.99),
        "peak_bytes": st["bytes_peak"],
        "result_bytes_reserved": res_est, "result_bytes_actual": res_act,
        "result_bytes_reserved_without_hints": no_hint_reserved,
        "jobs_under_reserved": under,
        "gen_s": round(t_gen, 1), "load_sweep": sweep, "longest_jobs": slow,
        "device_free_gb_at_start": round(free0 / 1e9, 1),
        "device_total_gb": round(total0 / 1e9, 1),
        "note": "seeded sample of the 10,000 jobs (same distribution); inputs resident; results "
                "released as soon as each job is done; distinct_hint from the size predictor "
                "(two-fold: trained on the other half of the jobs); Poisson arrivals at load x "
                "capacity (capacity from a pass with every job submitted at once, after a "
                "warm-up pass); latency = completion - submission",
    }


def cpu_baseline(reads, offs, k, n_sample):
    """The oracle as it stands, on the first n_sample reads, with every core
    the process may use, and on one thread on a sixteenth of that."""
    import oracle
    cores, detail = host_cores()
    r_s, o_s = reads[:int(offs[n_sample])], offs[:n_sample + 1]
    w_s = oracle.valid_windows(r_s, o_s, k)
    tc = time.perf_counter()
    oracle.count(r_s, o_s, k, threads=cores)
    dt = time.perf_counter() - tc
    n_1 = max(1, n_sample // 16)
    r_1, o_1 = reads[:int(offs[n_1])], offs[:n_1 + 1]
    w_1 = oracle.valid_windows(r_1, o_1, k)
    tc = time.perf_counter()
    oracle.count(r_1, o_1, k, threads=1)
    dt1 = time.perf_counter() - tc
    return {"value": round(w_s / dt, 1), "unit": "k-mers/s", "cores": cores, "kind": "oracle",
            "sample": "first %d of %d reads of the headline workload (%d valid windows, k = %d), "
                      "oracle on %d threads, %.1f s" % (n_sample, offs.size - 1, w_s, k, cores, dt),
            "one_thread_value": round(w_1 / dt1, 1),
            "one_thread_sample": "first %d reads (%d valid windows)" % (n_1, w_1),
            "cpu_model": cpu_model(), "host_cores": detail}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", type=int, default=3, help="headline workload (3: 40M reads)")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--second-k-steps", type=int, default=10,
                    help="timed calls of the headline reads at the workload's second k (0: skip)")
    ap.add_argument("--cpu-sample-reads", type=int, default=16_000_000)
    ap.add_argument("--c2-steps", type=int, default=20,
                    help="timed calls on the 1,000,000-read workload (0: skip its legs)")
    ap.add_argument("--batched-sets", type=int, default=4096,
                    help="sets of the batched workload to run (0: skip the batched leg)")
    ap.add_argument("--batched-budget-gib", type=float, default=96.0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--served-jobs", type=int, default=500,
                    help="jobs of the served workload to run (0: skip the served leg)")
    ap.add_argument("--served-budget-gib", type=float, default=150.0)
    ap.add_argument("--served-workers", type=int, default=4)
    ap.add_argument("--served-load", type=float, default=0.7)
    ap.add_argument("--sort-steps", type=int, default=5,
                    help="calls of the sort-based leaf count to time (0: skip)")
    ap.add_argument("--fastq-steps", type=int, default=5,
                    help="calls of the FASTQ parser on the 1,000,000 reads as FASTQ text (0: skip)")
    ap.add_argument("--long-k", type=int, default=100,
                    help="k of the long-key leg (65..128: four-word keys)")
    ap.add_argument("--long-k-steps", type=int, default=3,
                    help="calls of the long-key leg to time (0: skip)")
    ap.add_argument("--stream-pieces", type=int, default=4,
                    help="pieces of the streamed leg: reads counted from host memory in pieces "
                         "whose results are merged (0: skip)")
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
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    cfg = synth.make_config(args.config)
    k = args.k or cfg["ks"][0]
    P = cfg["P"]
    reads, offs = cfg["reads"], cfg["offsets"]
    rt = torch.from_numpy(reads).to(dev)
    ot = torch.from_numpy(offs.view(np.int64)).to(dev)
    cap = kc.max_outputs(offs, k)
    words = kc.kc.key_words(k)
    keys = torch.empty((cap, words) if words > 1 else (cap,), dtype=torch.int64, device=dev)
    cnts = torch.empty(cap, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    print("bench: inputs ready in %.1fs (%d reads, %d bytes)" % (time.time() - t0, len(offs) - 1,
                                                                  reads.size),
          file=sys.stderr, flush=True)
    copy_gbs = copy_rate(torch, dev, args.copy_gib)
    ceil = kc.kc.measure_ceilings(4 << 30, stream)

    head = timed_steps(kc, torch, rt, ot, k, P, keys, cnts, cap, args.steps, args.warmup, stream)
    st = head["st"]
    W = st["valid_windows"]
    value = W / (head["ms_step"] / 1e3)
    roofline = roofline_of(head, k, cfg["name"], copy_gbs, ceil)
    roofline["ceilings"] = {n: (round(v, 2) if isinstance(v, float) else v)
                            for n, v in ceil.items()}
    print("bench: headline k=%d %.2f ms per call" % (k, head["ms_step"]), file=sys.stderr,
          flush=True)

    second = None
    k2s = [x for x in cfg["ks"] if x != k]
    if args.second_k_steps > 0 and k2s:
        k2 = k2s[0]
        r2 = timed_steps(kc, torch, rt, ot, k2, P, keys, cnts, cap, args.second_k_steps, 2,
                         stream)
        s2 = r2["st"]
        second = {"k": k2, "value": round(s2["valid_windows"] / (r2["ms_step"] / 1e3), 1),
                  "unit": "k-mers/s", "ms_per_step": round(r2["ms_step"], 4),
                  "ms_median": round(float(np.median(r2["step_ms"])), 4),
                  "valid_windows": s2["valid_windows"], "distinct": r2["n_out"],
                  "second_count_records": s2["second_records"],
                  "refined_leaves": s2["n_overflow"], "refined_records": s2["refined_records"],
                  "roofline": roofline_of(r2, k2, cfg["name"], copy_gbs, ceil)}
    t_h2d = h2d_ms(torch, dev, reads, offs)
    del rt, ot, keys, cnts
    kc.lib().kc_release_scratch()
    torch.cuda.empty_cache()

    # the 1,000,000-read workload: plain figure, sort-based leaves, FASTQ, pieces, long keys
    c2 = None
    if args.c2_steps > 0:
        cfg2 = synth.make_config(2)
        r2h, o2h = cfg2["reads"], cfg2["offsets"]
        k2 = 31
        rt = torch.from_numpy(r2h).to(dev)
        ot = torch.from_numpy(o2h.view(np.int64)).to(dev)
        cap2 = kc.max_outputs(o2h, k2)
        keys = torch.empty(cap2, dtype=torch.int64, device=dev)
        cnts = torch.empty(cap2, dtype=torch.int32, device=dev)
        r = timed_steps(kc, torch, rt, ot, k2, cfg2["P"], keys, cnts, cap2, args.c2_steps, 3,
                        stream)
        W2 = r["st"]["valid_windows"]
        c2 = {"workload": cfg2["name"], "k": k2, "P": cfg2["P"],
              "value": round(W2 / (r["ms_step"] / 1e3), 1), "unit": "k-mers/s",
              "ms_per_step": round(r["ms_step"], 4),
              "ms_median": round(float(np.median(r["step_ms"])), 4),
              "valid_windows": W2, "distinct": r["n_out"],
              "roofline": roofline_of(r, k2, cfg2["name"], copy_gbs, ceil)}
        if args.sort_steps > 0:
            # the paper's own counting step (sort + run-length accumulate of
            # each owner's records) on the same partitions, for comparison
            o1 = kc.options(timing=1, mode=1)
            kc.count_into(rt, ot, k2, cfg2["P"], keys, cnts, cap2, o1, stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            leaf1 = 0.0
            for _ in range(args.sort_steps):
                kc.count_into(rt, ot, k2, cfg2["P"], keys, cnts, cap2, o1, stream)
                leaf1 += kc.last_stats()["ms_stage"]["leaf_large"]
            torch.cuda.synchronize()
            ms1 = (time.perf_counter() - t1) * 1e3 / args.sort_steps
            c2["sort_mode"] = {"value": round(W2 / (ms1 / 1e3), 1), "unit": "k-mers/s",
                               "ms_per_step": round(ms1, 4),
                               "leaf_ms": round(leaf1 / args.sort_steps, 4),
                               "note": "kc_options.mode = 1: each leaf's records sorted in LDS "
                                       "and run-length accumulated"}
        if args.fastq_steps > 0:
            text = synth.to_fastq(r2h, o2h, seed=1)
            tt = torch.frombuffer(bytearray(text), dtype=torch.uint8).to(dev)
            del text
            pr, po, _ = kc.parse_fastx(tt)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.fastq_steps):
                pr, po, _ = kc.parse_fastx(tt)
            torch.cuda.synchronize()
            ms_p = (time.perf_counter() - t1) * 1e3 / args.fastq_steps
            ok = pr.numel() == r2h.size and po.numel() == o2h.size
            t1 = time.perf_counter()
            for _ in range(args.fastq_steps):
                pr, po, _ = kc.parse_fastx(tt)
                kc.count_into(pr, po, k2, cfg2["P"], keys, cnts, cap2, None, stream)
            torch.cuda.synchronize()
            ms_pc = (time.perf_counter() - t1) * 1e3 / args.fastq_steps
            c2["fastq"] = {"text_bytes": tt.numel(), "records": po.numel() - 1,
                           "parsed_whole": ok, "parse_ms": round(ms_p, 4),
                           "parse_gbs": round(tt.numel() / (ms_p / 1e3) / 1e9, 1),
                           "parse_and_count_ms": round(ms_pc, 4),
                           "from_text_value": round(W2 / (ms_pc / 1e3), 1), "unit": "k-mers/s"}
            del tt, pr, po
        if args.stream_pieces > 0:
            chunk = (r2h.size + args.stream_pieces - 1) // args.stream_pieces
            host_pinned = torch.from_numpy(r2h).pin_memory()
            kc.count_chunked(host_pinned, o2h, k2, cfg2["P"], chunk_bytes=chunk)
            torch.cuda.synchronize()
            reps = 3
            t1 = time.perf_counter()
            for _ in range(reps):
                sk_, sc_ = kc.count_chunked(host_pinned, o2h, k2, cfg2["P"], chunk_bytes=chunk)
            torch.cuda.synchronize()
            ms_s = (time.perf_counter() - t1) * 1e3 / reps
            c2["streamed"] = {"pieces": args.stream_pieces, "ms_per_step": round(ms_s, 4),
                              "value": round(W2 / (ms_s / 1e3), 1), "unit": "k-mers/s",
                              "same_distinct": int(sc_.numel()) == r["n_out"]}
            del sk_, sc_, host_pinned
        if args.long_k_steps > 0:
            kl = args.long_k
            cap_l = max(1, kc.max_outputs(o2h, kl))
            keys_l = torch.empty((cap_l, 4), dtype=torch.int64, device=dev)
            cnts_l = torch.empty(cap_l, dtype=torch.int32, device=dev)
            ol = kc.options(timing=1)
            kc.count_into(rt, ot, kl, cfg2["P"], keys_l, cnts_l, cap_l, ol, stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.long_k_steps):
                n_l = kc.count_into(rt, ot, kl, cfg2["P"], keys_l, cnts_l, cap_l, ol, stream)
            torch.cuda.synchronize()
            ms_l = (time.perf_counter() - t1) * 1e3 / args.long_k_steps
            st_l = kc.last_stats()
            c2["long_k"] = {"k": kl, "value": round(st_l["valid_windows"] / (ms_l / 1e3), 1),
                            "unit": "k-mers/s", "ms_per_step": round(ms_l, 4),
                            "distinct": n_l}
            del keys_l, cnts_l
        del rt, ot, keys, cnts
        kc.lib().kc_release_scratch()
        torch.cuda.empty_cache()
        print("bench: 1M-read legs done", file=sys.stderr, flush=True)

    batched = None
    if args.batched_sets > 0:
        batched = batched_leg(args.batched_sets, args.batched_budget_gib, not args.no_tune)
        kc.lib().kc_release_scratch()
        torch.cuda.empty_cache()

    served = None
    if args.served_jobs > 0:
        served = served_leg(args.served_jobs, args.served_budget_gib, args.served_workers,
                            args.served_load)
        kc.lib().kc_release_scratch()
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(reads, offs, k, min(args.cpu_sample_reads, len(offs) - 1))

    line = {
        "metric": METRIC,
        "value": round(value, 1), "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms_step"], 4),
        "ms_median": round(float(np.median(head["step_ms"])), 4),
        "ms_best": round(min(head["step_ms"]), 4),
        "h2d_ms": round(t_h2d, 4),
        "end_to_end_value": round(W / ((head["ms_step"] + t_h2d) / 1e3), 1),
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if k <= 32 else "u128",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "k": k, "P": P, "reads": len(offs) - 1,
                   "read_len": 150, "valid_windows": W, "distinct": head["n_out"],
                   "second_count_records": st["second_records"],
                   "refined_leaves": st["n_overflow"], "refined_records": st["refined_records"],
                   "mode": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "second_k": second,
        "c2": c2,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
