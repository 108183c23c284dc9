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
           ("msda_fwd.hip", "msda_bwd.hip", "msda_tiles.hip", "msda_sort.hip", "msda_batch.hip",
            "msda_util.hip", "msda_vis.hip", "msda_softmax.hip", "msda_noalloc.hip",
            "msda_api.cpp")]
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


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    return res.returncode, out


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libmsda.so (always recompiles): one
    object per source, compiled in parallel, then one link."""
    import shutil
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    tmpdir = tempfile.mkdtemp(prefix="msda_build_")
    try:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]
        cflags = [f for f in FLAGS if f != "-shared"]
        cmds = [[HIPCC] + cflags + ["-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(_run, cmds))
        for (rc, out), src in zip(results, SOURCES):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({rc}):\n{out}")
            if verbose and out:
                print(out)
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        rc, out = _run(link)
        if rc != 0:
            raise RuntimeError(f"link failed ({rc}):\n{out}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
