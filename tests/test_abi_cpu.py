"""C-ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and its host-only helpers behave."""
import ctypes
import os
import re

import numpy as np

import paper_2505_04431_amd as kc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc))
                   if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kc_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    L = kc.lib()
    syms = header_symbols()
    assert "kc_count" in syms and "kc_count_ex" in syms
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(kc.EXPORTED_SYMBOLS) == syms


def test_library_is_gfx950_build():
    assert kc.lib().kc_version().decode().endswith("gfx950")
    with open(kc.library_path(), "rb") as f:
        blob = f.read()
    assert b"gfx950" in blob


def test_max_outputs_and_strerror():
    offs = np.array([0, 5, 5, 7, 100], dtype=np.uint64)
    assert kc.max_outputs(offs, 3) == 3 + 0 + 0 + 91
    assert kc.max_outputs(offs, 1) == 100
    assert kc.max_outputs(np.array([0, 5, 3], dtype=np.uint64), 2) == 0
    L = kc.lib()
    assert L.kc_strerror(0) == b"ok"
    assert L.kc_strerror(-3) == b"output capacity too small"
    assert L.kc_strerror(-99) == b"unknown status"


def test_options_layout_matches_header():
    # kc_options: 11 ints + 1 reserved; kc_stats: 13 uint64 + 13 doubles
    assert ctypes.sizeof(kc.kc.KcOptions) == 12 * 4
    assert ctypes.sizeof(kc.kc.KcStats) == 13 * 8 + 13 * 8


def test_struct_layouts_match_c_compiler(tmp_path):
    """sizeof/offsetof of every public struct, as gcc lays out include/kc.h,
    equal the ctypes mirrors of the binding."""
    mirrors = {"kc_options": kc.kc.KcOptions, "kc_stats": kc.kc.KcStats,
               "kc_job_info": kc.kc.KcJobInfo, "kc_serve_stats": kc.kc.KcServeStats,
               "kc_ceilings": kc.kc.KcCeilings, "kc_batch_wave": kc.kc.KcBatchWave}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kc.h"', '#include "kc_bench.h"',
             "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in mirrors.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(py, fname).offset, (cname, fname)
