"""Canonical k-mer counting on one MI355X (gfx950), HIP kernels behind a C ABI.

The Python layer only marshals arguments: every step of the counting path runs
in ``libkc.so``. Importing works without a GPU (so the library can be loaded and
inspected on a build host); calls need a ROCm device and raise otherwise.
"""
from .kc import (FASTA, FASTQ, FASTX_AUTO, BatchPlan, KcError, Predictor, Server,  # noqa: F401
                 count, count_chunked, count_into, count_noalloc_into, filter_min_count, last_stats, lib,
                 library_path, max_outputs, merge_counts, options, parse_fastx, spectrum,
                 EXPORTED_SYMBOLS, STATUS)

__all__ = ["BatchPlan", "Predictor", "Server", "count", "spectrum", "filter_min_count",
           "merge_counts", "count_chunked", "parse_fastx", "FASTX_AUTO", "FASTQ", "FASTA",
           "count_into", "count_noalloc_into", "max_outputs", "last_stats", "options", "KcError", "lib",
           "library_path", "EXPORTED_SYMBOLS", "STATUS"]
