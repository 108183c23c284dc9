"""Launch-shape autotuner for the MSDA kernels.

A launch shape ("tile") is the work order (anchor or view, see
include/msda.h), the number of waves per anchor (anchor order) or per
workgroup (view order), and the number of channels each lane owns (which
fixes how many samples a wave processes at once). The best choice depends on the problem: anchors and
cameras set the parallelism, the feature dtype the load width. For a given
workload the tuner runs every shape the library accepts, checks that its
results agree with the library's own choice (a shape that disagrees is
dropped, never timed), times the survivors with HIP events on the launch
stream, and caches the fastest per pass in a JSON file keyed by device
architecture, feature dtype and a shape bucket.

    tiles = autotune.tune_single(feat, layout, loc, w, grad_out)   # tunes and caches
    ops.forward(feat, layout, loc, w, tile=tiles["forward"])
    ops.forward(feat, layout, loc, w, tile="auto")                 # cached lookup

The cache lives at $MSDA_TUNE_CACHE, else ~/.cache/msda/tune.json.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional

import torch

CACHE_ENV = "MSDA_TUNE_CACHE"
WAVES = (1, 2, 4, 8)
CPL = {torch.float32: (4, 2, 1), torch.bfloat16: (8, 4, 2), torch.float16: (8, 4, 2),
       torch.float8_e4m3fn: (16, 8, 4), torch.uint8: (16, 8, 4)}
_DTYPE_NAME = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16",
               torch.float8_e4m3fn: "fp8",
               torch.uint8: "fp8"}


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "msda",
                                                     "tune.json")


def _pow2_bucket(n: int) -> int:
    b = 1
    while b < n:
        b <<= 1
    return b


def _arch() -> str:
    if torch.cuda.is_available():
        props = torch.cuda.get_device_properties(0)
        return getattr(props, "gcnArchName", props.name).split(":")[0]
    return "cpu"


def shape_key(dtype, C, G, L, P, cams, anchors, batch=1, kind="single", arch=None) -> str:
    """Cache key: arch, dtype, channels, groups, levels, keypoints and
    power-of-two buckets of the cameras and of batch x anchors."""
    return "/".join(str(x) for x in (
        arch or _arch(), kind, _DTYPE_NAME.get(dtype, str(dtype)), f"C{C}", f"G{G}", f"L{L}",
        f"P{P}", f"N{_pow2_bucket(cams)}", f"A{_pow2_bucket(max(1, batch * anchors))}"))


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(entries: Dict[str, dict], path: Optional[str] = None) -> str:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    merged = load_cache(path)
    merged.update(entries)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(merged, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def lookup(key: str, path: Optional[str] = None) -> Optional[dict]:
    return load_cache(path).get(key)


ORDERS = ("anchor", "view")


def candidates(dtype, C: int, G: int, orders=ORDERS) -> List[dict]:
    """Launch shapes the library accepts for C channels in G groups: C/cpl a
    power of two <= 64 and whole lanes per group, in each work order."""
    out = []
    for order in orders:
        for cpl in CPL[dtype]:
            lps = C // cpl if C % cpl == 0 else 0
            cpg = C // G
            if (not lps or lps & (lps - 1) or lps > 64 or cpg % cpl or
                    (cpg // cpl) & (cpg // cpl - 1)):
                continue
            for w in WAVES:
                out.append({"waves_per_anchor": w, "chans_per_lane": cpl, "order": order})
    return out


def _time(fn, reps: int) -> float:
    """Median milliseconds of fn() over reps, HIP events on the current stream."""
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def _agree(x: torch.Tensor, ref: torch.Tensor, tol: float) -> bool:
    x, ref = x.double(), ref.double()
    den = float(torch.linalg.vector_norm(ref))
    num = float(torch.linalg.vector_norm(x - ref))
    return bool(torch.isfinite(x).all()) and num <= tol * max(den, 1e-30)


def tune_single(feat, layout, loc, w, grad_out=None, level_scale=None, reps: int = 5,
                save: bool = True, path: Optional[str] = None) -> dict:
    """Tune the single-call forward (and backward when grad_out is given)."""
    from . import ops
    B, R, C = feat.shape
    A, P, N = loc.shape[1], loc.shape[2], loc.shape[3]
    L, G = w.shape[4], w.shape[5]
    key = shape_key(feat.dtype, C, G, L, P, N, A, B, "single")
    result = {"key": key}
    ref_out = ops.forward(feat, layout, loc, w, level_scale=level_scale)
    best = None
    for t in candidates(feat.dtype, C, G):
        out = ops.forward(feat, layout, loc, w, level_scale=level_scale, tile=t)
        if not _agree(out, ref_out, 1e-5):
            continue
        ms = _time(lambda: ops.forward(feat, layout, loc, w, level_scale=level_scale, tile=t), reps)
        if best is None or ms < best[1]:
            best = (t, ms)
    result["forward"], result["forward_ms"] = best
    if grad_out is not None and feat.dtype in (torch.float32, torch.bfloat16, torch.float16):
        ws = torch.empty(ops.backward_workspace_bytes(feat, layout, loc, w) + 256,
                         dtype=torch.uint8, device=feat.device)
        ref = ops.backward(feat, layout, loc, w, grad_out, workspace=ws)
        ref = [r.clone() for r in ref]
        best = None
        for t in candidates(feat.dtype, C, G):
            got = ops.backward(feat, layout, loc, w, grad_out, tile=t, workspace=ws)
            tol = 1e-2 if feat.dtype in (torch.bfloat16, torch.float16) else 1e-4
            if not all(_agree(g, r, tol) for g, r in zip(got, ref)):
                continue
            ms = _time(lambda: ops.backward(feat, layout, loc, w, grad_out, tile=t, workspace=ws),
                       reps)
            if best is None or ms < best[1]:
                best = (t, ms)
        result["backward"], result["backward_ms"] = best
    if save:
        save_cache({key: {k: v for k, v in result.items() if k != "key"}}, path)
    return result


def tune_batch(batch, reps: int = 3, save: bool = True, path: Optional[str] = None) -> dict:
    """Tune a SceneBatch: the same launch shape serves its forward and
    backward; the fastest for forward + backward is kept and left set."""
    cams = max(layout.num_cams for _, layout, _, _ in batch.scenes)
    anchors = sum(loc.shape[0] for _, _, loc, _ in batch.scenes)
    key = shape_key(batch.dtype, batch.C, batch.G, batch.L, batch.P, cams, anchors, 1, "batch")
    batch.set_tile(None)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    ref = [t.clone() for t in batch.out + [g for g in batch.grad_feat if g is not None]]
    best = None
    tol = 1e-2 if batch.dtype in (torch.bfloat16, torch.float16) else 1e-4
    for t in candidates(batch.dtype, batch.C, batch.G, orders=("anchor", "view")):
        batch.set_tile(t)
        batch.forward()
        batch.backward()
        torch.cuda.synchronize()
        got = batch.out + [g for g in batch.grad_feat if g is not None]
        if not all(_agree(g, r, tol) for g, r in zip(got, ref) if r.numel()):
            continue
        ms = _time(lambda: (batch.forward(), batch.backward()), reps)
        if best is None or ms < best[1]:
            best = (t, ms)
    batch.set_tile(best[0])
    result = {"key": key, "tile": best[0], "step_ms": best[1]}
    if save:
        save_cache({key: {"tile": best[0], "step_ms": best[1]}}, path)
    return result
