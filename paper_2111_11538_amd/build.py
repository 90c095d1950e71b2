"""Build the gfx950 HIP library ``libpf.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpf.so")
SOURCES = [os.path.join(HERE, "csrc", "pf_api.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         # keep the compiler from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, out: str | None = None, extra: tuple = ()) -> str:
    """Compile ``libpf.so`` (or, with `out`, another copy of it; `extra`
    appends flags, such as host-pass sanitizers)."""
    lib = out or LIB
    cmd = [HIPCC] + FLAGS + list(extra) + ["-o", lib + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
