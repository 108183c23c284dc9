#!/usr/bin/env python3
"""Benchmark of the MSDA hot path on one MI355X.

One step = the whole hot path over one batch: the forward kernel and the
backward (grad_feat, grad_sampling_loc, grad_weights) on the 64-camera scene
(64 cameras, 4 levels from a 256x448 image, C=256 in 8 groups, 900 anchors x
13 keypoints), BF16 feature storage with FP32 arithmetic. Inputs are seeded
synthetic tensors already resident in HBM when timing starts.

Prints one JSON line: GSamples/s of forward+backward (one sample = one
bilinear interpolation of all C channels at one (anchor, keypoint, camera,
level)), the FP32-storage rate beside it, a roofline object for the dominant
kernel (algorithmic bytes per launch / its event-timed duration, against the
8 TB/s HBM peak) and the FP64 CPU oracle's rate on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cam64", choices=["cam64", "train16", "sparse4d"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage comparison")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 12-scene batched form (graph-replayed, autotuned)")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-cache steps (1 GiB write before each step)")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 forward")
    ap.add_argument("--no-f16", action="store_true", help="skip the FP16-storage comparison")
    ap.add_argument("--no-softmax", action="store_true",
                    help="skip the steps with weights generated from logits")
    ap.add_argument("--no-visible", action="store_true",
                    help="skip the projection + visible-view steps (outside-in camera network)")
    ap.add_argument("--no-autograd", action="store_true",
                    help="skip the 16-camera training step through the autograd Function")
    ap.add_argument("--cpu-anchors", type=int, default=0,
                    help="anchors in the oracle's timed sample (0 = all of them)")
    return ap.parse_args()


def bytes_per_sample(C, G, L, P, N, s):
    """Bytes one sample accesses, per pass, counting every corner access (the
    effective gather traffic: caches serve most re-reads, so this is not HBM
    traffic): 4 corner rows of C elements of s bytes, the sample's G weights,
    its share of the location (shared by L levels) and of the anchor's output
    row (shared by P*N*L samples). The backward re-reads the corners, scatters
    4 corner contributions at the feature's precision, reads weights and
    writes their gradient, reads the location and writes its gradient, and
    reads grad_out."""
    share_out = C * 4.0 / (P * N * L)
    fwd = 4 * C * s + G * 4 + 8.0 / L + share_out
    bwd = 4 * C * s + 4 * C * s + 2 * G * 4 + 2 * 8.0 / L + share_out
    return fwd, bwd


def footprint_bytes(p, s):
    """Unique bytes each pass must move through HBM at least (every tensor
    read or written once): the HBM roofline's algorithmic bytes. Per unit:
    s bytes per feature element (B*R*C of them), 4*G per sample for the
    weights (and 4*G for grad_weights), 8 per (anchor, keypoint, camera)
    for the location (and 8 for its gradient), 4*C per anchor for out or
    grad_out. By kernel: the forward gather reads feat, weights and locations
    and writes out; the backward gather reads feat, weights, locations and
    grad_out and writes grad_weights and grad_sampling_loc; the grad_feat
    reduction reads weights and grad_out and writes grad_feat."""
    B, A, P, N, L = p.batch, p.num_anchors, p.num_points, p.num_cams, p.num_levels
    C, G = p.channels, p.groups
    S = B * A * P * N * L
    feat = B * int(p.rows) * C * s
    w = S * G * 4
    loc = B * A * P * N * 8
    row = B * A * C * 4
    terms = {
        "fwd": {"feat": feat, "weights": w, "loc": loc, "out": row},
        "bwd_gather": {"feat": feat, "weights": w, "grad_weights": w, "loc": loc,
                       "grad_loc": loc, "grad_out": row},
        "gfeat": {"grad_feat": feat, "weights": w, "grad_out": row},
    }
    return {k: (sum(v.values()), v) for k, v in terms.items()}


KERNEL_PASS = {"msda_fwd_kernel": "fwd", "msda_fwd_view_kernel": "fwd",
               "msda_bwd_kernel": "bwd_gather", "msda_bwd_view_kernel": "bwd_gather",
               "gfeat_tile_kernel": "gfeat", "gfeat_tile_kernel_coarse": "gfeat"}


class HipEvents:
    """hipEvent_t pairs through the HIP runtime torch has already loaded."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        if self.hip.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def destroy(self, e):
        self.hip.hipEventDestroy(e)

    def record(self, e):
        """Record on torch's current stream (the stream the library launches on)."""
        import torch
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        if self.hip.hipEventRecord(e, stream) != 0:
            raise RuntimeError("hipEventRecord failed")


def kernel_source_hash():
    """Hash of the library sources (the counters are void once they change)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_10819_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, dtype: str):
    """(HBM bytes per launch, L2 hit rate) from a committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None, None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        table = json.load(open(path))
    except (OSError, ValueError):
        return None, None
    ent = table.get(f"{kernel}/{workload}/{dtype}")
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None, None
    return ent.get("hbm_bytes_per_launch"), ent.get("l2_hit_rate")


def run_gpu(args, torch, ops, synth, p, feat_dtype, steps, warmup, cold=False, weights=None,
            logits=False, graph=False):
    """Time `steps` forward+backward steps. Every kernel the library launches
    is bracketed by HIP events on its stream (the library's benchmark hook),
    so per-kernel average durations come from the timed region itself.
    weights: instead of the workload's (e.g. logits, with logits=True)."""
    lib = ops._lib.load()
    dev = "cuda"
    feat = p.feat.to(feat_dtype).to(dev)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index, dev)
    loc = p.sampling_loc.to(dev)
    w = (weights if weights is not None else p.weights).to(dev)
    go = synth.grad_out_like(p, seed=1).to(dev)
    out = torch.empty(p.batch, p.num_anchors, p.channels, device=dev)
    ws_bytes = ops.backward_workspace_bytes(feat, layout, loc, w, logits=logits)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev) if ws_bytes else None
    fws_bytes = ops.forward_workspace_bytes(feat, layout, loc, w, logits=logits)
    fws = torch.empty(fws_bytes + 256, dtype=torch.uint8, device=dev) if fws_bytes else None

    def fwd():
        ops.forward(feat, layout, loc, w, out=out, workspace=fws, logits=logits)

    def bwd():
        ops.backward(feat, layout, loc, w, go, workspace=ws, logits=logits)

    def step():
        fwd()
        bwd()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    ev = HipEvents()
    cap = 32                                       # kernels recorded per step

    def instrumented(n, only=None):
        """n steps with the library's kernels bracketed by events (all of
        them, or only the kernel named `only`), plus stream events around
        each step's forward and backward calls. Returns the per-kernel
        durations and the steps' (start, after forward, end) events."""
        lib.msda_set_kernel_event_filter(only.encode() if only else None)
        arrays, names, marks = [], [], []
        for _ in range(n):
            arr = (ctypes.c_void_p * (2 * cap))()
            for i in range(2 * cap):
                arr[i] = ev.create()
            arrays.append(arr)
            marks.append((ev.create(), ev.create(), ev.create()))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            ops._lib.check(lib.msda_set_kernel_events(arrays[i], cap))
            ev.record(marks[i][0])
            fwd()
            ev.record(marks[i][1])
            bwd()
            ev.record(marks[i][2])
            k = lib.msda_recorded_kernels()
            names.append([lib.msda_recorded_kernel_name(j).decode() for j in range(k)])
            ops._lib.check(lib.msda_set_kernel_events(None, 0))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.msda_set_kernel_event_filter(None)
        per_kernel = {}
        for arr, nm in zip(arrays, names):
            for j, name in enumerate(nm):
                per_kernel.setdefault(name, []).append(ev.elapsed_ms(arr[2 * j], arr[2 * j + 1]))
        steps_ms = [ev.elapsed_ms(a, c) for a, _, c in marks]
        fwd_ms = [ev.elapsed_ms(a, b) for a, b, _ in marks]
        for arr in arrays:
            for e in arr:
                ev.destroy(e)
        for m in marks:
            for e in m:
                ev.destroy(e)
        return t1 - t0, per_kernel, steps_ms, fwd_ms

    # Per-kernel durations from a short instrumented pass outside the timed
    # region (an event pair around every launch costs about 10% of a step),
    # which also names the dominant kernel (largest time per step).
    probe = max(2, min(steps, 5))
    _, pk, _, _ = instrumented(probe)
    kern = {n: {"ms": sum(v) / len(v), "per_step": len(v) / probe} for n, v in pk.items()}
    dominant = max(kern, key=lambda n: kern[n]["ms"] * kern[n]["per_step"])
    # The timed region: events only around the dominant kernel's launches
    # (its average duration for the roofline) and around each step's calls.
    total_s, pk, steps_ms, fwd_ms = instrumented(steps, only=dominant)
    dl = pk.get(dominant, [])
    res = {"total_s": total_s, "kernels": kern, "probe_steps": probe,
           "timed_kernel": {"name": dominant, "ms": sum(dl) / len(dl) if dl else None,
                            "per_step": len(dl) / steps},
           "step_ms": pct(steps_ms), "fwd_ms": pct(fwd_ms),
           "bwd_ms": pct([a - b for a, b in zip(steps_ms, fwd_ms)])}
    if cold:
        # the same steps with the caches cold: a 1 GiB write (twice the
        # memory-side cache) before each, outside the events
        flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        cold_ms = []
        a, b = ev.create(), ev.create()
        for _ in range(steps):
            flush.fill_(1.0)
            ev.record(a)
            step()
            ev.record(b)
            torch.cuda.synchronize()
            cold_ms.append(ev.elapsed_ms(a, b))
        ev.destroy(a)
        ev.destroy(b)
        del flush
        res["cold_ms"] = pct(cold_ms)
    if graph:
        res["graph"] = graph_step(torch, ops, feat, layout, loc, w, go, out, fws, ws, logits,
                                  steps, warmup)
    return res


def graph_step(torch, ops, feat, layout, loc, w, go, out, fws, ws, logits, steps, warmup):
    """The same forward + backward step captured once in a HIP graph and
    replayed (no launch gaps between the library's kernels). Each replay's
    outputs are checked against an eager step's, bit for bit, with eager work
    between replays; a capture the runtime refuses is reported, not fatal."""
    def step():
        ops.forward(feat, layout, loc, w, out=out, workspace=fws, logits=logits)
        return ops.backward(feat, layout, loc, w, go, workspace=ws, logits=logits)

    eager = step()
    ref = [out.clone()] + [t.clone() for t in eager]
    torch.cuda.synchronize()
    try:
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(g, stream=stream):
                grads = step()
        torch.cuda.current_stream().wait_stream(stream)
        same = True
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            same = same and all(torch.equal(a, b) for a, b in zip([out] + list(grads), ref))
            step()                                  # eager work between replays
            torch.cuda.synchronize()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return {"ms_per_step": round(dt / steps * 1e3, 4), "replays_equal_eager": bool(same),
                "note": "fwd+bwd captured once (torch.cuda.graph) and replayed; not the headline"}
    except RuntimeError as e:
        return {"error": str(e)[:200]}




def pct(v):
    """median, p10 and p90 of a list of milliseconds."""
    import numpy as np
    a = np.asarray(v, dtype=np.float64)
    return {"median": round(float(np.median(a)), 4), "p10": round(float(np.percentile(a, 10)), 4),
            "p90": round(float(np.percentile(a, 90)), 4)}


def run_fp8_forward(torch, ops, p, steps, warmup):
    """The FP8 precision form's forward (per-level scales; the quantiser runs
    once, outside the timing), event-timed per call."""
    dev = "cuda"
    layout = ops.Layout(p.spatial_shapes, p.level_start_index, dev)
    codes, scale = ops.quantize_fp8(p.feat.to(dev), layout)
    loc, w = p.sampling_loc.to(dev), p.weights.to(dev)
    out = torch.empty(p.batch, p.num_anchors, p.channels, device=dev)
    fws = ops.forward_workspace_bytes(codes, layout, loc, w)
    ws = torch.empty(fws + 256, dtype=torch.uint8, device=dev) if fws else None
    for _ in range(warmup):
        ops.forward(codes, layout, loc, w, level_scale=scale, out=out, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ops.forward(codes, layout, loc, w, level_scale=scale, out=out, workspace=ws)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return pct(times)


def run_batched(torch, ops, synth, steps, warmup):
    """The uneven 12-scene batch (BF16 storage) in the batched form: launch
    shape from the autotuner (tuned here, not cached), forward + backward
    captured once in a HIP graph and replayed `steps` times; the eager rate of
    the same calls beside it."""
    from paper_2601_10819_amd import autotune
    probs = synth.batched(seed=0)
    scenes = [(p.feat[0].to(torch.bfloat16).cuda(), ops.Layout(p.spatial_shapes, p.level_start_index),
               p.sampling_loc[0].cuda(), p.weights[0].cuda()) for p in probs]
    batch = ops.SceneBatch(scenes)
    gen = torch.Generator(device="cuda").manual_seed(3)
    for go in batch.grad_out:
        go.normal_(generator=gen)
    tuned = autotune.tune_batch(batch, reps=3, save=False)

    def step():
        batch.forward()
        batch.backward()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            step()
    torch.cuda.current_stream().wait_stream(stream)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - t0
    S = batch.samples
    return {
        "workload": "batch_12scenes_uneven",
        "scenes": [[p.num_cams, int(p.rows), p.num_anchors] for p in probs],
        "samples_per_step": S,
        "tile": tuned["tile"],
        "graph_ms_per_step": round(graph_s / steps * 1e3, 4),
        "graph_value": round(S * steps / graph_s / 1e9, 4),
        "eager_ms_per_step": round(eager_s / steps * 1e3, 4),
        "eager_value": round(S * steps / eager_s / 1e9, 4),
        "unit": "GSamples/s",
    }


def run_visible(torch, ops, synth, p, steps, warmup, fused=False):
    """The 64-camera pyramid (BF16) with the sampling locations produced by
    the projection step from an outside-in camera network (anchors seen by
    a fraction of the cameras): one step = projection + visible-view forward
    + backward, timed with stream events (per-kernel durations from a few
    instrumented steps with the library's HIP-event hook). fused:
    the visibility-weighted fusion form (seeded positive view scores), with
    the score gradient."""
    lib = ops._lib.load()
    dev = "cuda"
    g = synth.outside_in(seed=0, cams=p.num_cams, anchors=p.num_anchors, P=p.num_points)
    anchors, keypoints = g.anchors.to(dev), g.keypoints.to(dev)
    projection, image_hw = g.projection.to(dev), g.image_hw.to(dev)
    feat = p.feat.to(torch.bfloat16).to(dev)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index, dev)
    w = p.weights.to(dev)
    go = synth.grad_out_like(p, seed=1).to(dev)
    out = torch.empty(p.batch, p.num_anchors, p.channels, device=dev)
    loc, vis = ops.project_keypoints(anchors, keypoints, projection, image_hw, g.dt)
    d = ops.make_desc(feat, layout, loc, w)
    fws = torch.empty(int(lib.msda_forward_visible_workspace_size(ctypes.byref(d))) + 256,
                      dtype=torch.uint8, device=dev)
    bws = torch.empty(int(lib.msda_backward_visible_workspace_size(ctypes.byref(d))) + 256,
                      dtype=torch.uint8, device=dev)
    gen = torch.Generator().manual_seed(2)
    score = (torch.rand(vis.shape, generator=gen) + 0.05).to(dev)

    def step():
        l, v = ops.project_keypoints(anchors, keypoints, projection, image_hw, g.dt)
        if fused:
            ops.forward_fused(feat, layout, l, w, v, score, out=out, workspace=fws)
            ops.backward_fused(feat, layout, l, w, v, score, out, go, workspace=bws)
        else:
            ops.forward_visible(feat, layout, l, w, v, out=out, workspace=fws)
            ops.backward_visible(feat, layout, l, w, v, go, workspace=bws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = HipEvents()
    # per-kernel durations from a few instrumented steps (an event pair
    # around every launch), then the timed steps with stream events only
    cap = 40
    per_kernel = {}
    arr = (ctypes.c_void_p * (2 * cap))()
    for i in range(2 * cap):
        arr[i] = ev.create()
    for _ in range(3):
        ops._lib.check(lib.msda_set_kernel_events(arr, cap))
        step()
        k = lib.msda_recorded_kernels()
        names = [lib.msda_recorded_kernel_name(j).decode() for j in range(k)]
        ops._lib.check(lib.msda_set_kernel_events(None, 0))
        torch.cuda.synchronize()
        for j, name in enumerate(names):
            per_kernel.setdefault(name, []).append(ev.elapsed_ms(arr[2 * j], arr[2 * j + 1]))
    for e in arr:
        ev.destroy(e)
    marks = [(ev.create(), ev.create()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in marks:
        ev.record(a)
        step()
        ev.record(b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps_ms = [ev.elapsed_ms(a, b) for a, b in marks]
    for a, b in marks:
        ev.destroy(a)
        ev.destroy(b)
    frac = float(vis.float().mean())
    S = p.samples
    st = pct(steps_ms)
    return {
        "workload": "scene_64cam_outside_in" + ("_fused" if fused else ""),
        "visible_pair_fraction": round(frac, 4),
        "visible_samples_per_step": int(round(S * frac)),
        "step_ms": st,
        "wall_ms_per_step": round((t1 - t0) / steps * 1e3, 4),
        "value_visible": round(S * frac / (st["median"] * 1e-3) / 1e9, 4),
        "value_nominal": round(S / (st["median"] * 1e-3) / 1e9, 4),
        "unit": "GSamples/s (visible samples / nominal B*A*P*N*L samples per step time)",
        "kernels_ms": {n: round(sum(v) / len(v), 4) for n, v in per_kernel.items()},
    }


def run_autograd(torch, ops, synth, steps, warmup):
    """The outside-in training step of the 16-camera workload (B = 2, 4
    levels from 384x640, C = 256 in 8 groups, 1800 anchors x 13 keypoints,
    BF16 features, FP32 locations and weights, 25% of keypoints outside each
    camera's view) through the autograd Function: out = msda(feat, loc, w),
    then out.backward(grad_out), the leaves' .grad cleared (set to None)
    before each step as an optimizer's zero_grad does. Wall clock over the
    steps; stream events split each step's forward and backward."""
    p = synth.train16()
    dev = "cuda"
    feat = p.feat.to(torch.bfloat16).to(dev).requires_grad_(True)
    loc = p.sampling_loc.to(dev).requires_grad_(True)
    w = p.weights.to(dev).requires_grad_(True)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index, dev)
    go = synth.grad_out_like(p, seed=1).to(dev)
    ev = HipEvents()

    def step(marks=None):
        feat.grad = loc.grad = w.grad = None
        if marks:
            ev.record(marks[0])
        out = ops.msda(feat, layout, loc, w)
        if marks:
            ev.record(marks[1])
        out.backward(go)
        if marks:
            ev.record(marks[2])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    marks = [(ev.create(), ev.create(), ev.create()) for _ in range(steps)]
    t0 = time.perf_counter()
    for m in marks:
        step(m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = [ev.elapsed_ms(a, c) for a, _, c in marks]
    fw = [ev.elapsed_ms(a, b) for a, b, _ in marks]
    for m in marks:
        for e in m:
            ev.destroy(e)
    S = p.samples
    ms = (t1 - t0) / steps * 1e3
    return {"workload": p.name, "batch": p.batch, "cameras": p.num_cams,
            "anchors": p.num_anchors, "samples_per_step": S,
            "ms_per_step": round(ms, 4), "value": round(S / (ms * 1e-3) / 1e9, 4),
            "unit": "GSamples/s", "step_ms": pct(st), "fwd_ms": pct(fw),
            "bwd_ms": pct([a - b for a, b in zip(st, fw)]),
            "note": "BF16 features; torch.autograd.Function forward + backward (all three "
                    "gradients), grads set to None before each step"}


def copy_bandwidth(torch, ops, nbytes=1 << 30, reps=10):
    """Achievable streaming bandwidth (read + write) of the library's copy kernel."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    ops.stream_copy(dst, src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ops.stream_copy(dst, src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return 2 * nbytes / dt / 1e9


def cpu_baseline(p, anchors, min_seconds=10.0, max_reps=20):
    """The FP64 oracle (as it stands) on the first `anchors` anchors of the
    same workload, forward + full backward on BF16-widened features, repeated
    until about `min_seconds` of CPU time have been measured."""
    import numpy as np
    import torch
    import oracle
    oracle._load()
    sub_loc = p.sampling_loc[:, :anchors].contiguous()
    sub_w = p.weights[:, :anchors].contiguous()
    feat = p.feat.to(torch.bfloat16).double().numpy()
    go = np.random.default_rng(0).standard_normal((p.batch, anchors, p.channels))
    reps, dt = 0, 0.0
    while reps < max_reps and (reps == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        oracle.forward(feat, p.spatial_shapes, p.level_start_index, sub_loc, sub_w)
        oracle.backward(feat, p.spatial_shapes, p.level_start_index, sub_loc, sub_w, go)
        dt += time.perf_counter() - t0
        reps += 1
    samples = p.batch * anchors * p.num_points * p.num_cams * p.num_levels
    return samples * reps / dt / 1e9, dt, oracle.num_threads(), samples, reps


def cpu_baselines(synth, min_seconds=3.0, max_reps=50):
    """The FP64 oracle (as it stands) on the smaller workloads, in full:
    forward alone and forward + full backward, each repeated until about
    `min_seconds` have been measured. A baseline only."""
    import numpy as np
    import oracle
    oracle._load()
    res = {}
    for maker in (synth.tiny, lambda: synth.sparse4d(seed=0), synth.train16):
        p = maker()
        feat = p.feat.double().numpy()
        go = np.random.default_rng(0).standard_normal((p.batch, p.num_anchors, p.channels))
        row = {"samples": p.samples}
        for name in ("fwd", "fwd_bwd"):
            reps, dt = 0, 0.0
            while reps < max_reps and (reps == 0 or dt < min_seconds):
                t0 = time.perf_counter()
                oracle.forward(feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights)
                if name == "fwd_bwd":
                    oracle.backward(feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                                    p.weights, go)
                dt += time.perf_counter() - t0
                reps += 1
            row[name + "_s"] = round(dt / reps, 5)
            row[name + "_GSamples_per_s"] = round(p.samples * reps / dt / 1e9, 6)
        res[p.name] = row
    res["cores"] = oracle.num_threads()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the MSDA path "
              "here is single-GPU; camera sharding across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2601_10819_amd import ops, synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ops._lib.load()

    maker = {"cam64": synth.cam64, "train16": synth.train16,
             "sparse4d": lambda: synth.sparse4d(seed=0)}[args.workload]
    p = maker()
    S = p.samples
    print(f"# workload {p.name} {p.dims()} samples/step {S}", file=sys.stderr, flush=True)

    bf = run_gpu(args, torch, ops, synth, p, torch.bfloat16, args.steps, args.warmup,
                 cold=not args.no_cold, graph=True)
    print(f"# bf16 done: {bf}", file=sys.stderr, flush=True)
    ms_step = bf["total_s"] / args.steps * 1e3
    value = S * args.steps / bf["total_s"] / 1e9

    fp = None
    if not args.no_fp32:
        fp = run_gpu(args, torch, ops, synth, p, torch.float32, args.steps, args.warmup)
        print(f"# fp32 done: {fp}", file=sys.stderr, flush=True)
    hf = None
    if not args.no_f16:
        hf = run_gpu(args, torch, ops, synth, p, torch.float16, args.steps, args.warmup)
        print(f"# f16 done: {hf}", file=sys.stderr, flush=True)

    C, G, L, P, N = p.channels, p.groups, p.num_levels, p.num_points, p.num_cams
    fwd_b, bwd_b = bytes_per_sample(C, G, L, P, N, 2)
    # roofline of the dominant kernel (largest time per step): its
    # algorithmic bytes are the unique bytes its pass must move through HBM
    # (footprint_bytes), over its average launch duration in the timed region
    ks = bf["kernels"]
    kern = bf["timed_kernel"]["name"]
    kms = bf["timed_kernel"]["ms"]
    fpb = footprint_bytes(p, 2)
    kpass = KERNEL_PASS.get(kern)
    kbytes, kterms = fpb[kpass] if kpass else (None, None)
    achieved = kbytes / (kms * 1e-3) / 1e9 if kbytes else None
    traffic, l2hit = measured_traffic(kern, p.name, "bf16")
    # the same launch counted per corner access (every re-read included)
    per_access = {"fwd": fwd_b, "bwd_gather": bwd_b - 4 * C * 2, "gfeat": 4 * C * 2}.get(kpass)
    step_fp = fpb["fwd"][0] + fpb["bwd_gather"][0] + fpb["gfeat"][0]

    res = {
        "metric": "MSDA fwd+bwd GSamples/s (64-camera scene, BF16 storage, FP32 math)",
        "value": round(value, 4),
        "unit": "GSamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": p.name, "batch": p.batch, "cameras": N, "levels": L,
                   "level_shapes": [list(map(int, s)) for s in p.spatial_shapes[0].tolist()],
                   "channels": C, "groups": G, "anchors": p.num_anchors, "keypoints": P,
                   "samples_per_step": S},
        "step_ms": bf["step_ms"],
        "fwd_ms": bf["fwd_ms"],
        "bwd_ms": bf["bwd_ms"],
        "kernels_ms": {n: round(v["ms"], 4) for n, v in ks.items()},
        "kernels_note": (f"average per launch from {bf['probe_steps']} instrumented steps outside "
                         "the timed region (an event pair around every launch); inside it only "
                         "the roofline kernel is bracketed"),
        "headline_note": ("value: K back-to-back steps (warm caches) on the wall clock; "
                          "cold.value: the same step with L2 and the memory-side cache "
                          "evicted before each step (event-timed median)"),
        # the whole step's unique bytes (each tensor once per pass) per step
        # time, against HBM peak; and its bytes counted per corner access
        # (caches serve re-reads, so that rate is not bounded by HBM)
        "footprint_hbm_frac_fwd_bwd": round(step_fp / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "effective_access_TBps_fwd_bwd": round(S * (fwd_b + bwd_b) / (ms_step * 1e-3) / 1e12, 3),
        "roofline": {"bound": "hbm", "kernel": kern,
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic,
                     "alg_bytes_per_launch": int(kbytes) if kbytes else None,
                     "alg_bytes_terms": kterms,
                     "avg_launch_ms": round(kms, 4),
                     "traffic_GBps": round(traffic / (kms * 1e-3) / 1e9, 1) if traffic else None,
                     "l2_hit_rate": l2hit,
                     "effective_gather_GBps": (round(S * per_access / (kms * 1e-3) / 1e9, 1)
                                               if per_access else None)},
    }
    if "graph" in bf:
        res["graph"] = bf["graph"]
    if "cold_ms" in bf:
        res["cold"] = {"ms_per_step": bf["cold_ms"],
                       "value": round(S / (bf["cold_ms"]["median"] * 1e-3) / 1e9, 4),
                       "note": "1 GiB written before each step, outside its events"}
    if fp is not None:
        fp_ms = fp["total_s"] / args.steps * 1e3
        res["fp32_ms_per_step"] = round(fp_ms, 4)
        res["fp32_value"] = round(S * args.steps / fp["total_s"] / 1e9, 4)
        res["bf16_speedup_vs_fp32"] = round(fp_ms / ms_step, 3)
        res["fp32_kernels_ms"] = {n: round(v["ms"], 4) for n, v in fp["kernels"].items()}
        res["fp32_fwd_ms"] = fp["fwd_ms"]
        res["fp32_bwd_ms"] = fp["bwd_ms"]
    if hf is not None:
        hf_ms = hf["total_s"] / args.steps * 1e3
        res["f16"] = {"ms_per_step": round(hf_ms, 4),
                      "value": round(S * args.steps / hf["total_s"] / 1e9, 4),
                      "fwd_ms": hf["fwd_ms"], "bwd_ms": hf["bwd_ms"],
                      "kernels_ms": {n: round(v["ms"], 4) for n, v in hf["kernels"].items()},
                      "note": "IEEE half storage, FP32 arithmetic (the paper's own precision)"}
        if fp is not None:
            res["f16"]["speedup_vs_fp32"] = round(fp["total_s"] / hf["total_s"], 3)
    if not args.no_softmax:
        g = torch.Generator().manual_seed(3)
        x = torch.randn(p.weights.shape, generator=g) * 2.0
        sm = {}
        for name, xt in (("f32_logits", x), ("bf16_logits", x.to(torch.bfloat16))):
            r = run_gpu(args, torch, ops, synth, p, torch.bfloat16, args.steps, args.warmup,
                        weights=xt, logits=True)
            sm[name] = {"ms_per_step": round(r["total_s"] / args.steps * 1e3, 4),
                        "value": round(S * args.steps / r["total_s"] / 1e9, 4),
                        "fwd_ms": r["fwd_ms"], "bwd_ms": r["bwd_ms"],
                        "kernels_ms": {n: round(v["ms"], 4) for n, v in r["kernels"].items()}}
            print(f"# softmax {name} done: {sm[name]}", file=sys.stderr, flush=True)
        sm["note"] = ("BF16 features, weights generated inside from per-group logits "
                      "(softmax over keypoints x cameras x levels); grad_weights = gradient "
                      "of the logits")
        res["softmax_weights"] = sm
    if not args.no_fp8:
        f8 = run_fp8_forward(torch, ops, p, args.steps, args.warmup)
        res["fp8_forward"] = {"ms": f8, "value": round(S / (f8["median"] * 1e-3) / 1e9, 4),
                              "unit": "GSamples/s (forward only)"}
    if not args.no_visible:
        res["visible"] = run_visible(torch, ops, synth, p, args.steps, args.warmup)
        print(f"# visible done: {res['visible']}", file=sys.stderr, flush=True)
        res["visible_fused"] = run_visible(torch, ops, synth, p, args.steps, args.warmup,
                                           fused=True)
        print(f"# fused done: {res['visible_fused']}", file=sys.stderr, flush=True)
    if not args.no_batched:
        res["batched"] = run_batched(torch, ops, synth, args.steps, args.warmup)
        print(f"# batched done: {res['batched']}", file=sys.stderr, flush=True)
    if not args.no_autograd:
        res["autograd_train16"] = run_autograd(torch, ops, synth, args.steps, args.warmup)
        print(f"# autograd done: {res['autograd_train16']}", file=sys.stderr, flush=True)
    res["copy_GBps"] = round(copy_bandwidth(torch, ops), 1)

    if not args.no_cpu:
        anchors = args.cpu_anchors or p.num_anchors
        v, dt, cores, ns, reps = cpu_baseline(p, anchors)
        res["cpu_baseline"] = {"value": round(v, 6), "unit": "GSamples/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{p.name} anchors[0:{anchors}] ({ns} samples), FP64 "
                                         f"forward + full backward, {reps} runs in {dt:.1f} s"}
        res["cpu_baseline_configs"] = cpu_baselines(synth)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
