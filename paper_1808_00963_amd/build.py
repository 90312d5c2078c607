"""Builds libss.so (HIP, gfx950) in place."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libss.so")
SOURCES = ["ss_kernels.hip", "ss_merge.hip", "ss_sa.hip", "ss_api.cpp"]
ARCH = os.environ.get("SS_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        # no packed FP32 instructions anywhere in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"),
    ]


# Per-source extra flags.  The level kernels loop over their items (work
# counts are read on the device); LLVM's machine-level loop-invariant code
# motion would hoist dozens of thread-index-derived LDS addresses out of those
# loops and keep them live for the whole kernel, costing the occupancy the
# one-item bodies reach (e.g. the scatter 56 -> 84 VGPRs, one work group per
# compute unit instead of two).  Without it the addresses are computed where
# they are used.
EXTRA = {"ss_kernels.hip": ["-mllvm", "-disable-machine-licm"]}


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles every HIP source into libss.so (always recompiles when force)."""
    if not force and os.path.exists(LIB):
        return LIB
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="ss_build_") as d:
        objs = []
        for src in SOURCES:
            obj = os.path.join(d, src + ".o")
            cmd = [hipcc, *hipcc_flags(), *EXTRA.get(src, []), "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            subprocess.check_call(cmd)
            objs.append(obj)
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
