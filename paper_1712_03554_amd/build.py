"""Build libsframe.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import glob
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


# The host code (circuit loading and expansion, planning, serving, readout)
# built with UndefinedBehaviorSanitizer; device code is compiled as usual.
# Every report aborts the process.  The function and vptr checks are left
# out: the allocator hook is a foreign (ctypes) function pointer.
UBSAN_OUT = os.path.join(HERE, "libsframe_ubsan.so")


def _ubsan_libdir() -> str:
    """Directory of the shared UBSan runtime of hipcc's clang."""
    for d in sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux"), reverse=True):
        if os.path.exists(os.path.join(d, "libclang_rt.ubsan_standalone-x86_64.so")):
            return d
    return "/opt/rocm/llvm/lib/clang/22/lib/linux"


UBSAN_LIBDIR = os.environ.get("UBSAN_LIBDIR") or _ubsan_libdir()
UBSAN_FLAGS = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize=function,vptr",
               "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
               "-shared-libsan", "-Wl,-rpath," + UBSAN_LIBDIR]


def build(verbose: bool = False, timers: bool = False, out: str = OUT, ubsan: bool = False) -> str:
    """timers=True compiles in the tableau-track phase counters (profiling
    builds); ubsan=True builds the host code with UBSan (into UBSAN_OUT
    unless out is given)."""
    if ubsan and out == OUT:
        out = UBSAN_OUT
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ([HIPCC] + FLAGS + (["-DSF_TRACK_TIMERS"] if timers else []) + (UBSAN_FLAGS if ubsan else []) +
           ["-o", tmp, SRC])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
