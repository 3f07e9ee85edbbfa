"""Build the HIP library ``libkc.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libkc.so")
SOURCES = ["kc_kernels.hip", "kc_runtime.cpp", "kc_server.cpp", "kc_pred.hip", "kc_ceiling.hip", "kc_post.hip",
           "kc_parse.hip"]
HEADERS = ["kc_internal.h", "kc_host.h", "kc_sched.h", os.path.join("..", "..", "include", "kc.h")]
ARCH = os.environ.get("KC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def flags() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            # no packed fp32 instructions anywhere in the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile every source into libkc.so (always recompiles)."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + flags()
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                        and "warning: unknown" not in l.lower() or "error" in l.lower())
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
        if verbose and err.strip():
            print(err, file=sys.stderr)
        objs.append(obj)
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, SO)
    for o in objs:
        os.remove(o)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
