"""Build libmsda.so (the HIP kernels and the C ABI) in-tree with hipcc for gfx950.

    python -m paper_2601_10819_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmsda.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("msda_fwd.hip", "msda_bwd.hip", "msda_sort.hip", "msda_batch.hip", "msda_util.hip",
            "msda_vis.hip", "msda_softmax.hip", "msda_api.cpp")]
HEADERS = [os.path.join(CSRC, "msda_internal.h"), os.path.join(CSRC, "msda_common.h"),
           os.path.join(CSRC, "msda_gather.h"),
           os.path.join(ROOT, "include", "msda.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # hardware float atomics (no compare-and-swap loops) for the grad_feat scatter
    "-munsafe-fp-atomics",
    # no packed-FP32 instructions: write plain scalar float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libmsda.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if verbose and out:
        print(out)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
