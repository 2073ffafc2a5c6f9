"""Build libsparrow.so (HIP, gfx950) in-tree.

Flags that matter for the results:
  -ffp-contract=off   no a*b+c fusion: every binary32 op is rounded as written,
                      which keeps grid indices and done flags exact
  -fhip-fp32-correctly-rounded-divide-sqrt
                      IEEE division and square root
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keep packed FP32 instructions out of the generated code
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsparrow.so")
SOURCES = [os.path.join(CSRC, "sparrow.hip"), os.path.join(CSRC, "sparrow_ring.hip"),
           os.path.join(CSRC, "sparrow_learner.hip"),
           os.path.join(CSRC, "sparrow_peaks.hip")]
HEADERS = [os.path.join(CSRC, "sparrow_device.h"), os.path.join(CSRC, "sparrow_qnet.h"),
           os.path.join(CSRC, "sparrow_mlp.h"), os.path.join(CSRC, "sparrow_ring_dev.h"),
           os.path.join(CSRC, "sparrow_host.h"),
           os.path.join(ROOT, "include", "sparrow.h")]
ARCH = "gfx950"


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    return "hipcc"


def flags(extra=()):
    return ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature",
            "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
            "-Wall", "-Wno-unused-function", *extra]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libsparrow.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *flags(), "-shared", "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def asm(out_dir: str) -> list[str]:
    """Device assembly of the library (for inspection of our own build)."""
    os.makedirs(out_dir, exist_ok=True)
    outs = []
    for src in SOURCES:
        stem = os.path.splitext(os.path.basename(src))[0]
        out = os.path.join(out_dir, f"{stem}-gfx950.s")
        subprocess.check_call([hipcc(), *flags(), "--cuda-device-only", "-S", "-o", out, src])
        outs.append(out)
    return outs


if __name__ == "__main__":
    build(verbose=True)
    if len(sys.argv) > 1 and sys.argv[1] == "asm":
        import tempfile
        print(asm(sys.argv[2] if len(sys.argv) > 2 else os.path.join(tempfile.gettempdir(), "sparrow_asm")))
