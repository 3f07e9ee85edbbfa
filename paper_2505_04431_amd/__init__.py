"""Canonical k-mer counting on one MI355X (gfx950), HIP kernels behind a C ABI.

The Python layer only marshals arguments: every step of the counting path runs
in ``libkc.so``. Importing works without a GPU (so the library can be loaded and
inspected on a build host); calls need a ROCm device and raise otherwise.
"""
from .kc import (BatchPlan, KcError, Predictor, Server, count, count_into, filter_min_count,  # noqa: F401,E501
                 last_stats, lib, library_path, max_outputs, options, spectrum, EXPORTED_SYMBOLS,
                 STATUS)

__all__ = ["BatchPlan", "Predictor", "Server", "count", "spectrum", "filter_min_count", "count_into", "max_outputs", "last_stats", "options",
           "KcError", "lib", "library_path", "EXPORTED_SYMBOLS", "STATUS"]
