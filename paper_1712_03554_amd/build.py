"""Build libsframe.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "api.hip")
OUT = os.path.join(HERE, "libsframe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # every floating-point operation rounded on its own (no fused
         # multiply-add contraction): the same expression gives the same bits
         # in every kernel it is inlined into
         "-ffp-contract=off",
         # keep packed fp32 instructions out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, timers: bool = False, out: str = OUT) -> str:
    """timers=True compiles in the tableau-track phase counters (profiling builds)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + (["-DSF_TRACK_TIMERS"] if timers else []) + ["-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
