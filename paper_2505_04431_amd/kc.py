"""ctypes binding of ``include/kc.h`` (argument marshalling only).

Torch is used for device memory and the current stream; nothing is computed
here. If ``libkc.so`` is missing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libkc.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "KC_OK", -1: "KC_E_INVAL", -2: "KC_E_NOMEM", -3: "KC_E_CAPACITY",
          -4: "KC_E_OVERFLOW", -5: "KC_E_DEVICE", -6: "KC_E_INTERNAL"}

EXPORTED_SYMBOLS = ["kc_count", "kc_count_ex", "kc_max_outputs", "kc_last_stats",
                    "kc_release_scratch", "kc_strerror", "kc_last_error", "kc_version",
                    "kc_batch_plan", "kc_batch_run", "kc_batch_max_outputs", "kc_batch_stats",
                    "kc_batch_free", "kc_server_create", "kc_server_submit", "kc_server_poll",
                    "kc_server_wait", "kc_server_result", "kc_server_result_copy",
                    "kc_server_job_info", "kc_server_release", "kc_server_stats",
                    "kc_server_destroy", "kc_pred_create", "kc_pred_num_params",
                    "kc_pred_get_params", "kc_pred_set_params", "kc_pred_get_grads",
                    "kc_pred_forward", "kc_pred_gradient", "kc_pred_adam_step", "kc_pred_free",
                    "kc_measure_ceilings", "kc_spectrum", "kc_filter_min_count",
                    "kc_merge_counts", "kc_parse_fastx", "kc_count_noalloc", "kc_batch_waves",
                    "kc_batch_wave_info", "kc_batch_run_wave"]

JOB_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class KcOptions(ctypes.Structure):
    _fields_ = [("shard_bits", ctypes.c_int), ("leaf_target", ctypes.c_int),
                ("leaf_attempt", ctypes.c_int), ("table_slots_log2", ctypes.c_int),
                ("check", ctypes.c_int), ("timing", ctypes.c_int), ("mode", ctypes.c_int),
                ("scatter_tile", ctypes.c_int), ("split_tile", ctypes.c_int),
                ("refine_bits", ctypes.c_int), ("preagg", ctypes.c_int),
                ("reserved", ctypes.c_int * 1)]


class KcStats(ctypes.Structure):
    _fields_ = [("n_bases", ctypes.c_uint64), ("valid_windows", ctypes.c_uint64),
                ("distinct", ctypes.c_uint64), ("n_leaves", ctypes.c_uint64),
                ("n_levels", ctypes.c_uint64), ("n_overflow", ctypes.c_uint64),
                ("max_leaf_windows", ctypes.c_uint64), ("max_owner_windows", ctypes.c_uint64),
                ("refined_records", ctypes.c_uint64), ("large_records", ctypes.c_uint64),
                ("large_distinct", ctypes.c_uint64), ("second_records", ctypes.c_uint64),
                ("second_distinct", ctypes.c_uint64), ("ms_total", ctypes.c_double),
                ("ms_stage", ctypes.c_double * 12)]


class KcJobInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("worker", ctypes.c_int),
                ("k", ctypes.c_int), ("n_bytes", ctypes.c_uint64),
                ("valid_windows", ctypes.c_uint64), ("distinct", ctypes.c_uint64),
                ("result_estimate_bytes", ctypes.c_uint64), ("result_bytes", ctypes.c_uint64),
                ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_end_ms", ctypes.c_double)]


class KcServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("submitted", "completed", "failed", "queued", "running", "valid_windows",
                 "budget", "bytes_in_use", "bytes_peak", "estimate_misses",
                 "result_bytes_reserved", "result_bytes_actual", "slab_bytes",
                 "unplaced")] + \
               [(n, ctypes.c_double) for n in
                ("latency_p50_ms", "latency_p99_ms", "wait_p50_ms", "wait_p99_ms", "busy_ms")]


class KcBatchWave(ctypes.Structure):
    _fields_ = [("first_set", ctypes.c_uint32), ("n_sets", ctypes.c_uint32),
                ("first_read", ctypes.c_uint64), ("n_reads", ctypes.c_uint64),
                ("first_byte", ctypes.c_uint64), ("n_bytes", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("n_classes", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class KcCeilings(ctypes.Structure):
    _fields_ = [("copy_gbs", ctypes.c_double), ("hbm_insert_gops", ctypes.c_double),
                ("mall_insert_gops", ctypes.c_double), ("lds_insert_gops", ctypes.c_double),
                ("hbm_table_bytes", ctypes.c_uint64), ("mall_table_bytes", ctypes.c_uint64),
                ("lost", ctypes.c_uint64)]


def measure_ceilings(table_bytes: int = 4 << 30, stream=None) -> dict:
    """kc_measure_ceilings: copy, HBM / cache / LDS insert rates on this device."""
    c = KcCeilings()
    st = lib().kc_measure_ceilings(int(table_bytes), ctypes.byref(c), stream)
    if st != 0:
        raise KcError(st, lib().kc_last_error().decode())
    return {n: getattr(c, n) for n, _ in KcCeilings._fields_}


STAGES = ["pack", "window_hist", "owner_scatter", "split_hist", "split_scatter", "leaf_small",
          "leaf_large", "out_offsets", "concat", "check", "refine", "leaf_second"]


class KcError(RuntimeError):
    def __init__(self, status: int, message: str, n_out: int = 0):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, message))
        self.status = status
        self.n_out = n_out


def library_path() -> str:
    return _SO


def lib():
    """Load libkc.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                raise ImportError("libkc.so not built: run __graft_entry__.build() "
                                  "(or python -m paper_2505_04431_amd._build)")
            L = ctypes.CDLL(_SO)
            p, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
            L.kc_count.restype = i32
            L.kc_count.argtypes = [p, p, u64, i32, i32, p, p, p]
            L.kc_count_ex.restype = i32
            L.kc_count_ex.argtypes = [p, p, u64, i32, i32, p, p, u64, p, p, p]
            L.kc_count_noalloc.restype = i32
            L.kc_count_noalloc.argtypes = [p, p, u64, i32, i32, p, p, u64, p, p, p]
            L.kc_max_outputs.restype = u64
            L.kc_max_outputs.argtypes = [p, u64, i32]
            L.kc_last_stats.restype = i32
            L.kc_last_stats.argtypes = [p]
            L.kc_release_scratch.restype = None
            L.kc_release_scratch.argtypes = []
            L.kc_strerror.restype = ctypes.c_char_p
            L.kc_strerror.argtypes = [i32]
            L.kc_last_error.restype = ctypes.c_char_p
            L.kc_last_error.argtypes = []
            L.kc_version.restype = ctypes.c_char_p
            L.kc_version.argtypes = []
            L.kc_batch_plan.restype = i32
            L.kc_batch_plan.argtypes = [p, p, p, ctypes.c_uint32, i32, u64, p, p]
            L.kc_batch_waves.restype = ctypes.c_uint32
            L.kc_batch_waves.argtypes = [p]
            L.kc_batch_wave_info.restype = i32
            L.kc_batch_wave_info.argtypes = [p, ctypes.c_uint32, p]
            L.kc_batch_run_wave.restype = i32
            L.kc_batch_run_wave.argtypes = [p, ctypes.c_uint32, p, p, p, p, u64, p, p, p]
            L.kc_batch_run.restype = i32
            L.kc_batch_run.argtypes = [p, p, p, p, p, u64, p, p, p]
            L.kc_batch_max_outputs.restype = u64
            L.kc_batch_max_outputs.argtypes = [p]
            L.kc_batch_stats.restype = i32
            L.kc_batch_stats.argtypes = [p, p]
            L.kc_batch_free.restype = None
            L.kc_batch_free.argtypes = [p]
            L.kc_server_create.restype = i32
            L.kc_server_create.argtypes = [u64, i32, p, p]
            L.kc_server_submit.restype = i32
            L.kc_server_submit.argtypes = [p, p, p, u64, i32, i32, u64, p]
            L.kc_server_poll.restype = i32
            L.kc_server_poll.argtypes = [p, u64, p]
            L.kc_server_wait.restype = i32
            L.kc_server_wait.argtypes = [p, u64, p]
            L.kc_server_result.restype = i32
            L.kc_server_result.argtypes = [p, u64, p, p, p]
            L.kc_server_result_copy.restype = i32
            L.kc_server_result_copy.argtypes = [p, u64, p, p, u64, p, p]
            L.kc_server_job_info.restype = i32
            L.kc_server_job_info.argtypes = [p, u64, p]
            L.kc_server_release.restype = i32
            L.kc_server_release.argtypes = [p, u64]
            L.kc_server_stats.restype = i32
            L.kc_server_stats.argtypes = [p, p]
            L.kc_server_destroy.restype = None
            L.kc_server_destroy.argtypes = [p]
            L.kc_pred_create.restype = i32
            L.kc_pred_create.argtypes = [i32, i32, u64, p]
            L.kc_pred_num_params.restype = u64
            L.kc_pred_num_params.argtypes = [p]
            for name in ("kc_pred_get_params", "kc_pred_set_params", "kc_pred_get_grads"):
                getattr(L, name).restype = i32
                getattr(L, name).argtypes = [p, p, u64]
            L.kc_pred_forward.restype = i32
            L.kc_pred_forward.argtypes = [p, p, u64, p, p]
            L.kc_pred_gradient.restype = i32
            L.kc_pred_gradient.argtypes = [p, p, p, u64, p, p]
            L.kc_pred_adam_step.restype = i32
            L.kc_pred_adam_step.argtypes = [p, ctypes.c_float, p]
            L.kc_pred_free.restype = None
            L.kc_pred_free.argtypes = [p]
            L.kc_measure_ceilings.restype = i32
            L.kc_measure_ceilings.argtypes = [u64, p, p]
            L.kc_spectrum.restype = i32
            L.kc_spectrum.argtypes = [p, u64, ctypes.c_uint32, p, p]
            L.kc_filter_min_count.restype = i32
            L.kc_filter_min_count.argtypes = [p, p, u64, i32, ctypes.c_uint32, p, p, p, p]
            L.kc_merge_counts.restype = i32
            L.kc_merge_counts.argtypes = [p, p, u64, p, p, u64, i32, p, p, p, p]
            L.kc_parse_fastx.restype = i32
            L.kc_parse_fastx.argtypes = [p, u64, i32, p, u64, p, u64, p, p, p, p]
            _lib = L
    return _lib


def options(**kw) -> KcOptions:
    o = KcOptions()
    for name, v in kw.items():
        setattr(o, name, int(v))
    return o


def max_outputs(host_offsets, k: int) -> int:
    off = np.ascontiguousarray(np.asarray(host_offsets), dtype=np.uint64)
    return int(lib().kc_max_outputs(off.ctypes.data, off.size - 1, k))


def last_stats() -> dict:
    s = KcStats()
    lib().kc_last_stats(ctypes.byref(s))
    d = {name: getattr(s, name) for name, _ in KcStats._fields_ if name != "ms_stage"}
    d["ms_stage"] = {n: s.ms_stage[i] for i, n in enumerate(STAGES)}
    return d


def key_words(k: int) -> int:
    """64-bit words per key: 1 (k <= 32), 2 (k <= 64), 4 (k <= 128)."""
    return 1 if k <= 32 else (2 if k <= 64 else 4)


def _key_shape(n: int, words: int):
    return (n, words) if words > 1 else (n,)


def _check_tensor(t, what, dtypes):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (ROCm) tensor" % what)
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s" % (what, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)


def _check_outputs(out_keys, out_counts, capacity: int, k: int) -> None:
    # the library writes up to capacity keys of key_words(k) words each: the
    # tensors must hold them (it cannot check raw pointers itself)
    if not 1 <= k <= 128:
        return  # the library refuses k itself
    if out_keys.numel() < capacity * key_words(k):
        raise ValueError("out_keys holds %d words; capacity %d at k = %d needs %d"
                         % (out_keys.numel(), capacity, k, capacity * key_words(k)))
    if out_counts.numel() < capacity:
        raise ValueError("out_counts holds %d counts; capacity is %d" % (out_counts.numel(), capacity))


def count_into(reads, offsets, k: int, P: int, out_keys, out_counts, capacity: int,
               opts: KcOptions | None = None, stream=None) -> int:
    """Call kc_count_ex on torch device tensors; returns the number of keys written.
    out_keys must hold capacity * key_words(k) int64 words, out_counts capacity
    counts (checked)."""
    import torch
    _check_tensor(reads, "reads", (torch.uint8,))
    _check_tensor(offsets, "offsets", (torch.int64, torch.uint64))
    _check_tensor(out_keys, "out_keys", (torch.int64, torch.uint64))
    _check_tensor(out_counts, "out_counts", (torch.int32, torch.uint32))
    _check_outputs(out_keys, out_counts, capacity, k)
    if stream is None:
        stream = torch.cuda.current_stream(reads.device).cuda_stream
    n_out = ctypes.c_uint64(0)
    with torch.cuda.device(reads.device):
        st = lib().kc_count_ex(reads.data_ptr(), offsets.data_ptr(), offsets.numel() - 1, k, P,
                               out_keys.data_ptr(), out_counts.data_ptr(), capacity,
                               ctypes.byref(n_out),
                               ctypes.byref(opts) if opts is not None else None, stream)
    if st != 0:
        raise KcError(st, lib().kc_last_error().decode(), int(n_out.value))
    return int(n_out.value)


def count_noalloc_into(reads, offsets, k: int, P: int, out_keys, out_counts, capacity: int,
                       opts: KcOptions | None = None, stream=None) -> int:
    """Call kc_count_noalloc (the allocation-free form: fixed device scratch,
    synchronous) on torch device tensors; returns the number of keys written
    (outputs checked as in count_into)."""
    import torch
    _check_tensor(reads, "reads", (torch.uint8,))
    _check_tensor(offsets, "offsets", (torch.int64, torch.uint64))
    _check_tensor(out_keys, "out_keys", (torch.int64, torch.uint64))
    _check_tensor(out_counts, "out_counts", (torch.int32, torch.uint32))
    _check_outputs(out_keys, out_counts, capacity, k)
    if stream is None:
        stream = torch.cuda.current_stream(reads.device).cuda_stream
    n_out = ctypes.c_uint64(0)
    with torch.cuda.device(reads.device):
        st = lib().kc_count_noalloc(reads.data_ptr(), offsets.data_ptr(), offsets.numel() - 1, k,
                                    P, out_keys.data_ptr(), out_counts.data_ptr(), capacity,
                                    ctypes.byref(n_out),
                                    ctypes.byref(opts) if opts is not None else None, stream)
    if st != 0:
        raise KcError(st, lib().kc_last_error().decode(), int(n_out.value))
    return int(n_out.value)


def count(reads, offsets, k: int, P: int = 1, opts: KcOptions | None = None, stream=None,
          capacity: int | None = None):
    """Count canonical k-mers of device reads.

    reads: uint8 CUDA tensor; offsets: int64 CUDA tensor of n_reads+1 offsets.
    Returns (keys, counts): int64 tensors [D] (k <= 32) or [D, w] with the w = 2
    (k <= 64) or 4 (k <= 128) words of a key, least significant first, and
    int32 counts [D] (bit patterns of uint64 / uint32).
    """
    import torch
    if capacity is None:
        # every window starts at its own byte of reads: no copy of the offsets
        # to the host (kc_max_outputs would need one) for a tighter bound
        capacity = reads.numel()
    capacity = max(1, int(capacity))
    words = key_words(k)
    keys = torch.empty(_key_shape(capacity, words), dtype=torch.int64,
                       device=reads.device)
    counts = torch.empty(capacity, dtype=torch.int32, device=reads.device)
    n = count_into(reads, offsets, k, P, keys, counts, capacity, opts, stream)
    return keys[:n], counts[:n]


def spectrum(counts, max_count: int = 1000, stream=None) -> np.ndarray:
    """kc_spectrum of a count array (CUDA int32/uint32 tensor): uint64[max_count + 1]."""
    import torch
    _check_tensor(counts, "counts", (torch.int32, torch.uint32))
    if stream is None:
        stream = torch.cuda.current_stream(counts.device).cuda_stream
    out = np.zeros(max_count + 1, dtype=np.uint64)
    st = lib().kc_spectrum(counts.data_ptr(), counts.numel(), max_count, out.ctypes.data, stream)
    if st != 0:
        raise KcError(st, lib().kc_last_error().decode())
    return out


def filter_min_count(keys, counts, k: int, min_count: int, stream=None):
    """kc_filter_min_count: the (keys, counts) pairs with count >= min_count."""
    import torch
    _check_tensor(keys, "keys", (torch.int64, torch.uint64))
    _check_tensor(counts, "counts", (torch.int32, torch.uint32))
    n = counts.numel()
    ok = torch.empty_like(keys) if n else keys
    oc = torch.empty_like(counts) if n else counts
    if stream is None:
        stream = torch.cuda.current_stream(counts.device).cuda_stream
    n_out = ctypes.c_uint64(0)
    st = lib().kc_filter_min_count(keys.data_ptr(), counts.data_ptr(), n, k, min_count,
                                   ok.data_ptr(), oc.data_ptr(), ctypes.byref(n_out), stream)
    if st != 0:
        raise KcError(st, lib().kc_last_error().decode())
    return ok[:n_out.value], oc[:n_out.value]


def merge_counts(a_keys, a_counts, b_keys, b_counts, k: int, stream=None):
    """kc_merge_counts of two results (CUDA tensors as count() returns them)."""
    import torch
    for t, nm in ((a_keys, "a_keys"), (b_keys, "b_keys")):
        _check_tensor(t, nm, (torch.int64, torch.uint64))
    for t, nm in ((a_counts, "a_counts"), (b_counts, "b_counts")):
        _check_tensor(t, nm, (torch.int32, torch.uint32))
    na, nb = a_counts.numel(), b_counts.numel()
    words = key_words(k)
    if a_keys.numel() != na * words or b_keys.numel() != nb * words:
        raise ValueError("keys must hold %d word(s) per count" % words)
    dev = a_counts.device
    n = max(1, na + nb)
    ok = torch.empty(_key_shape(n, words), dtype=torch.int64, device=dev)
    oc = torch.empty(n, dtype=torch.int32, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    n_out = ctypes.c_uint64(0)
    st = lib().kc_merge_counts(a_keys.data_ptr(), a_counts.data_ptr(), na, b_keys.data_ptr(),
                               b_counts.data_ptr(), nb, k, ok.data_ptr(), oc.data_ptr(),
                               ctypes.byref(n_out), stream)
    if st != 0:
        raise KcError(st, lib().kc_last_error().decode())
    return ok[:n_out.value], oc[:n_out.value]


FASTX_AUTO, FASTQ, FASTA = 0, 1, 2


def parse_fastx(text, fmt: int = FASTX_AUTO, stream=None):
    """kc_parse_fastx of a FASTQ / FASTA text in a CUDA uint8 tensor.
    Returns (reads uint8, offsets int64, format) on the text's device, ready
    for count()."""
    import torch
    _check_tensor(text, "text", (torch.uint8,))
    dev = text.device
    n = text.numel()
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    reads = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
    cap = n // 64 + 16
    while True:
        offs = torch.empty(cap + 1, dtype=torch.int64, device=dev)
        nr, nbase, fo = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_int(fmt)
        st = lib().kc_parse_fastx(text.data_ptr() if n else None, n, fmt, reads.data_ptr(), n,
                                  offs.data_ptr(), cap, ctypes.byref(nr), ctypes.byref(nbase),
                                  ctypes.byref(fo), stream)
        if st == -3 and nr.value > cap:
            cap = nr.value
            continue
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode())
        return reads[:nbase.value], offs[:nr.value + 1], fo.value


_chunk_local = threading.local()


def _chunk_staging(dev, pin_bytes: int, n_offs: int, dev_bytes: int) -> dict:
    """The calling thread's staging for count_chunked on dev: two pinned and two
    device buffers for reads and offsets, a side stream and two events, kept
    between calls and grown when a call needs more (a pinned allocation costs
    milliseconds)."""
    import torch
    cache = getattr(_chunk_local, "staging", None)
    if cache is None:
        cache = _chunk_local.staging = {}
    st = cache.get(dev.index)
    if st is None:
        st = cache[dev.index] = {"stream": torch.cuda.Stream(device=dev),
                                 "done": [torch.cuda.Event() for _ in range(2)],
                                 "pin_r": None, "pin_o": None, "dev_r": None, "dev_o": None}
    for e in st["done"]:
        e.synchronize()  # no copy of an earlier call still reads these buffers
    if st["pin_r"] is None or st["pin_r"][0].numel() < pin_bytes:
        st["pin_r"] = [torch.empty(pin_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
    if st["pin_o"] is None or st["pin_o"][0].numel() < n_offs:
        st["pin_o"] = [torch.empty(n_offs, dtype=torch.int64, pin_memory=True) for _ in range(2)]
    if st["dev_r"] is None or st["dev_r"][0].numel() < dev_bytes:
        st["dev_r"] = [torch.empty(dev_bytes, dtype=torch.uint8, device=dev) for _ in range(2)]
    if st["dev_o"] is None or st["dev_o"][0].numel() < n_offs:
        st["dev_o"] = [torch.empty(n_offs, dtype=torch.int64, device=dev) for _ in range(2)]
    return st


def count_chunked(host_reads, host_offsets, k: int, P: int = 1, chunk_bytes: int = 1 << 30,
                  opts: KcOptions | None = None):
    """Count reads held in host memory in pieces of about chunk_bytes, so the
    input may exceed device memory (the result must fit): each piece's result
    is merged into the running one (kc_merge_counts). Pieces are staged
    through two pinned host buffers: while piece i is counted, piece i + 1 is
    copied into pinned memory (a host thread) and on to the device (a side
    stream). host_reads: uint8 numpy array, or a pinned uint8 CPU tensor
    (then pieces are copied to the device straight from it, with no staging
    copy); host_offsets: uint64 numpy array of n_reads + 1 offsets. Returns
    (keys, counts) on the current device."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    offs = np.ascontiguousarray(host_offsets, dtype=np.uint64)
    pinned_in = isinstance(host_reads, torch.Tensor) and host_reads.is_pinned()
    reads = host_reads if pinned_in else np.asarray(host_reads, dtype=np.uint8)
    n_reads = offs.size - 1
    dev = torch.device("cuda", torch.cuda.current_device())
    words = key_words(k)
    keys = torch.empty(_key_shape(0, words), dtype=torch.int64, device=dev)
    counts = torch.empty(0, dtype=torch.int32, device=dev)
    # pieces: reads [r, e), at least one read, then as many as fit in chunk_bytes
    pieces = []
    r = 0
    while r < n_reads:
        limit = int(offs[r]) + max(1, int(chunk_bytes))
        e = int(np.searchsorted(offs, np.uint64(limit), side="right")) - 1
        e = min(n_reads, max(e, r + 1))
        pieces.append((r, e))
        r = e
    if not pieces:
        return keys, counts
    # output room of each piece: its windows of length k (kc_max_outputs over
    # the piece's host offsets)
    lib_ = lib()
    caps = [max(1, int(lib_.kc_max_outputs(offs[r:].ctypes.data, e - r, k))) for r, e in pieces]
    max_b = max(1, max(int(offs[e] - offs[r]) for r, e in pieces))
    max_r = max(e - r for r, e in pieces)
    st_ = _chunk_staging(dev, 1 if pinned_in else max_b, max_r + 1, max_b)
    pin_r, pin_o, dev_r, dev_o = st_["pin_r"], st_["pin_o"], st_["dev_r"], st_["dev_o"]
    copy_stream, done = st_["stream"], st_["done"]

    sizes = [None] * len(pieces)

    def stage(i):  # host thread: piece i into pinned buffer i % 2
        s = i % 2
        done[s].synchronize()  # the upload that last read this buffer has finished
        r0, r1 = pieces[i]
        b0, b1 = int(offs[r0]), int(offs[r1])
        if not pinned_in:
            np.copyto(pin_r[s].numpy()[:b1 - b0], reads[b0:b1])
        pin_o[s].numpy()[:r1 - r0 + 1] = (offs[r0:r1 + 1] - np.uint64(b0)).view(np.int64)
        sizes[i] = (b1 - b0, r1 - r0, b0)

    def upload(i):  # side stream: pinned buffer i % 2 -> device buffer i % 2
        s = i % 2
        nb, nr, b0 = sizes[i]
        src = reads[b0:b0 + nb] if pinned_in else pin_r[s][:nb]
        with torch.cuda.stream(copy_stream):
            dev_r[s][:nb].copy_(src, non_blocking=True)
            dev_o[s][:nr + 1].copy_(pin_o[s][:nr + 1], non_blocking=True)
            done[s].record(copy_stream)

    # piece i + 1 travels to the device while piece i is counted; piece i + 2
    # is staged into pinned memory meanwhile
    compute = torch.cuda.current_stream(dev)
    n = len(pieces)
    with ThreadPoolExecutor(max_workers=1) as ex:
        stage(0)
        upload(0)
        fut = ex.submit(stage, 1) if n > 1 else None
        for i in range(n):
            s = i % 2
            if i + 1 < n:
                fut.result()
                upload(i + 1)  # its device buffer was last read by piece i - 1, counted
            if i + 2 < n:
                fut = ex.submit(stage, i + 2)
            compute.wait_event(done[s])
            nb, nr, _ = sizes[i]
            pk, pc = count(dev_r[s][:max(nb, 1)], dev_o[s][:nr + 1], k, P, opts=opts,
                           capacity=caps[i])
            keys, counts = merge_counts(keys, counts, pk, pc, k) if counts.numel() else (pk, pc)
    return keys, counts


def _stats_dict(s: KcStats) -> dict:
    d = {name: getattr(s, name) for name, _ in KcStats._fields_ if name != "ms_stage"}
    d["ms_stage"] = {n: s.ms_stage[i] for i, n in enumerate(STAGES)}
    return d


class BatchPlan:
    """A planned batch of read sets (kc_batch_plan / kc_batch_run / kc_batch_run_wave).

    set_reads, set_bytes, ks: per set (host sequences). The reads of all sets
    are consecutive in one stream; set s has its own k (1..32). hbm_budget:
    device bytes a memory wave may hold (0: one wave for all sets).
    """

    def __init__(self, set_reads, set_bytes, ks, P: int = 1, opts: KcOptions | None = None,
                 hbm_budget: int = 0):
        self.set_reads = np.ascontiguousarray(set_reads, dtype=np.uint64)
        self.set_bytes = np.ascontiguousarray(set_bytes, dtype=np.uint64)
        self.ks = np.ascontiguousarray(ks, dtype=np.int32)
        self.n_sets = int(self.ks.size)
        self._h = ctypes.c_void_p()
        st = lib().kc_batch_plan(self.set_reads.ctypes.data, self.set_bytes.ctypes.data,
                                 self.ks.ctypes.data, self.n_sets, P, int(hbm_budget),
                                 ctypes.byref(opts) if opts is not None else None,
                                 ctypes.byref(self._h))
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode())
        self.max_outputs = int(lib().kc_batch_max_outputs(self._h))
        self.waves = [self.wave_info(w) for w in range(int(lib().kc_batch_waves(self._h)))]

    def wave_info(self, w: int) -> dict:
        info = KcBatchWave()
        st = lib().kc_batch_wave_info(self._h, w, ctypes.byref(info))
        if st != 0:
            raise KcError(st, "wave %d" % w)
        return {n: getattr(info, n) for n, _ in KcBatchWave._fields_ if n != "pad"}

    def run_into(self, reads, offsets, out_keys, out_counts, capacity: int, stream=None):
        """Run every wave on device tensors of the whole batch; returns
        (n_pairs, set_offsets as a numpy uint64 array of n_sets + 1)."""
        import torch
        _check_tensor(reads, "reads", (torch.uint8,))
        _check_tensor(offsets, "offsets", (torch.int64, torch.uint64))
        if stream is None:
            stream = torch.cuda.current_stream(reads.device).cuda_stream
        set_off = np.zeros(self.n_sets + 1, dtype=np.uint64)
        n_out = ctypes.c_uint64(0)
        with torch.cuda.device(reads.device):
            st = lib().kc_batch_run(self._h, reads.data_ptr(), offsets.data_ptr(),
                                    out_keys.data_ptr(), out_counts.data_ptr(), capacity,
                                    set_off.ctypes.data, ctypes.byref(n_out), stream)
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode(), int(n_out.value))
        return int(n_out.value), set_off

    def run_wave_into(self, w: int, reads, offsets, out_keys, out_counts, capacity: int,
                      stream=None):
        """Run wave w on device tensors holding only that wave's reads and
        their offsets; returns (n_pairs, the wave's n_sets + 1 set offsets)."""
        import torch
        _check_tensor(reads, "reads", (torch.uint8,))
        _check_tensor(offsets, "offsets", (torch.int64, torch.uint64))
        if stream is None:
            stream = torch.cuda.current_stream(reads.device).cuda_stream
        set_off = np.zeros(self.waves[w]["n_sets"] + 1, dtype=np.uint64)
        n_out = ctypes.c_uint64(0)
        with torch.cuda.device(reads.device):
            st = lib().kc_batch_run_wave(self._h, w, reads.data_ptr(), offsets.data_ptr(),
                                         out_keys.data_ptr(), out_counts.data_ptr(), capacity,
                                         set_off.ctypes.data, ctypes.byref(n_out), stream)
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode(), int(n_out.value))
        return int(n_out.value), set_off

    def run(self, reads, offsets, stream=None):
        import torch
        cap = max(1, self.max_outputs)
        keys = torch.empty(cap, dtype=torch.int64, device=reads.device)
        counts = torch.empty(cap, dtype=torch.int32, device=reads.device)
        n, set_off = self.run_into(reads, offsets, keys, counts, cap, stream)
        return keys[:n], counts[:n], set_off

    def stats(self) -> dict:
        s = KcStats()
        lib().kc_batch_stats(self._h, ctypes.byref(s))
        return _stats_dict(s)

    def close(self):
        if self._h:
            lib().kc_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server (kc_server_*): jobs counted side by side on the device
    under a byte budget; results stay on the device until released.

    Inputs of a submitted job must stay alive (and unchanged) until the job
    has finished; this wrapper keeps a reference to them until release().
    """

    def __init__(self, budget_bytes: int, workers: int = 4, opts: KcOptions | None = None):
        self._h = ctypes.c_void_p()
        self._inputs = {}
        st = lib().kc_server_create(int(budget_bytes), int(workers),
                                    ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(self._h))
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode())

    def _chk(self, st):
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode())

    def submit(self, reads, offsets, k: int, P: int = 1, distinct_hint: int = 0) -> int:
        import torch
        _check_tensor(reads, "reads", (torch.uint8,))
        _check_tensor(offsets, "offsets", (torch.int64, torch.uint64))
        jid = ctypes.c_uint64(0)
        self._chk(lib().kc_server_submit(self._h, reads.data_ptr(), offsets.data_ptr(),
                                         offsets.numel() - 1, k, P, int(distinct_hint),
                                         ctypes.byref(jid)))
        self._inputs[jid.value] = (reads, offsets)
        return int(jid.value)

    def poll(self, job: int) -> str:
        s = ctypes.c_int(0)
        self._chk(lib().kc_server_poll(self._h, job, ctypes.byref(s)))
        return JOB_STATES[s.value]

    def wait(self, job: int) -> str:
        s = ctypes.c_int(0)
        self._chk(lib().kc_server_wait(self._h, job, ctypes.byref(s)))
        return JOB_STATES[s.value]

    def info(self, job: int) -> dict:
        i = KcJobInfo()
        self._chk(lib().kc_server_job_info(self._h, job, ctypes.byref(i)))
        d = {n: getattr(i, n) for n, _ in KcJobInfo._fields_}
        d["state"] = JOB_STATES[d["state"]]
        return d

    def result(self, job: int, stream=None):
        """Copy of a finished job's (keys, counts) as new device tensors."""
        import torch
        self.wait(job)
        info = self.info(job)
        n, words = int(info["distinct"]), key_words(info["k"])
        dev = torch.device("cuda", torch.cuda.current_device())
        keys = torch.empty(_key_shape(max(n, 1), words), dtype=torch.int64, device=dev)
        counts = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        n_out = ctypes.c_uint64(0)
        self._chk(lib().kc_server_result_copy(self._h, job, keys.data_ptr(), counts.data_ptr(),
                                              max(n, 1), ctypes.byref(n_out), stream))
        return keys[:n_out.value], counts[:n_out.value]

    def release(self, job: int):
        self._chk(lib().kc_server_release(self._h, job))
        self._inputs.pop(job, None)

    def stats(self) -> dict:
        s = KcServeStats()
        self._chk(lib().kc_server_stats(self._h, ctypes.byref(s)))
        return {n: getattr(s, n) for n, _ in KcServeStats._fields_}

    def close(self):
        if self._h:
            lib().kc_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._inputs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Predictor:
    """The device perceptron of kc_pred_* (forward, gradient, Adam step).

    Inputs are fp32 CUDA tensors: x [batch, n_features], targets [batch]."""

    def __init__(self, n_features: int, hidden: int = 32, seed: int = 1):
        self._h = ctypes.c_void_p()
        st = lib().kc_pred_create(n_features, hidden, seed, ctypes.byref(self._h))
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode())
        self.n_features, self.hidden = n_features, hidden
        self.n_params = int(lib().kc_pred_num_params(self._h))

    def _chk(self, st):
        if st != 0:
            raise KcError(st, lib().kc_last_error().decode())

    def _x(self, x):
        import torch
        _check_tensor(x, "x", (torch.float32,))
        if x.dim() != 2 or x.shape[1] != self.n_features:
            raise ValueError("x must be [batch, %d]" % self.n_features)

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._chk(lib().kc_pred_get_params(self._h, out.ctypes.data, self.n_params))
        return out

    def set_params(self, values):
        v = np.ascontiguousarray(values, dtype=np.float32)
        if v.size != self.n_params:
            raise ValueError("expected %d parameters" % self.n_params)
        self._chk(lib().kc_pred_set_params(self._h, v.ctypes.data, self.n_params))

    def grads(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._chk(lib().kc_pred_get_grads(self._h, out.ctypes.data, self.n_params))
        return out

    def forward(self, x, stream=None):
        import torch
        self._x(x)
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        self._chk(lib().kc_pred_forward(self._h, x.data_ptr(), x.shape[0], y.data_ptr(), stream))
        return y

    def gradient(self, x, target, want_loss: bool = True, stream=None):
        import torch
        self._x(x)
        _check_tensor(target, "target", (torch.float32,))
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        loss = ctypes.c_float(0.0)
        self._chk(lib().kc_pred_gradient(self._h, x.data_ptr(), target.data_ptr(), x.shape[0],
                                         ctypes.byref(loss) if want_loss else None, stream))
        return float(loss.value) if want_loss else None

    def adam_step(self, lr: float, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(torch.cuda.current_device()).cuda_stream
        self._chk(lib().kc_pred_adam_step(self._h, ctypes.c_float(lr), stream))

    def close(self):
        if self._h:
            lib().kc_pred_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
