"""Shared test helpers: moving synthetic problems to the device, error
metrics, and oracle evaluation on anchor subsets."""
from __future__ import annotations

import numpy as np
import torch

# Bars (per-tensor normwise error ||x - ref|| / ||ref||, which equals
# RMS(err) / RMS(ref)): FP32 forward 1e-5, FP32 gradients 1e-4, BF16 storage
# 1e-2 of the output RMS, each against the FP64 oracle.
FWD_F32_TOL = 1e-5
GRAD_F32_TOL = 1e-4
BF16_TOL = 1e-2
# Largest single-element error allowed, relative to the reference RMS; catches
# an isolated wrong element that a norm over many elements would average away.
FWD_F32_MAXREL = 2e-4
GRAD_F32_MAXREL = 2e-3


def normwise(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    return float(num / den) if den > 0 else float(num)


def maxrel(x, ref) -> float:
    """max |x - ref| / RMS(ref)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    err = np.abs(x - ref).max() if ref.size else 0.0
    return float(err / rms) if rms > 0 else float(err)


def assert_close(x, ref, tol, maxtol=None, what=""):
    nw = normwise(x, ref)
    assert nw <= tol, f"{what}: normwise error {nw:.3e} > {tol:.1e}"
    if maxtol is not None:
        mr = maxrel(x, ref)
        assert mr <= maxtol, f"{what}: max error / RMS {mr:.3e} > {maxtol:.1e}"
    return nw


def host(t) -> np.ndarray:
    return t.detach().float().cpu().double().numpy() if t.dtype == torch.bfloat16 else \
        t.detach().cpu().double().numpy()


def to_device(p, feat_dtype=torch.float32, device="cuda"):
    """(feat, layout, loc, w) on the device; feat cast with round-to-nearest-even."""
    from paper_2601_10819_amd import ops
    feat = p.feat.to(feat_dtype).to(device)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index, device)
    return feat, layout, p.sampling_loc.to(device), p.weights.to(device)


def anchor_subset(p, count, seed=0):
    """A seeded sorted subset of anchor indices (all when count >= A)."""
    A = p.num_anchors
    if count >= A:
        return np.arange(A)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(A, size=count, replace=False))


def oracle_forward_subset(oracle, feat64, p, idx):
    """Oracle out[:, idx] (every anchor is independent in the forward)."""
    return oracle.forward(feat64, p.spatial_shapes, p.level_start_index,
                          p.sampling_loc[:, idx].contiguous(), p.weights[:, idx].contiguous())


def oracle_backward_subset(oracle, feat64, p, idx, grad_out):
    """Oracle grad_loc and grad_w at anchors idx (per-anchor quantities)."""
    _, gl, gw = oracle.backward(feat64, p.spatial_shapes, p.level_start_index,
                                p.sampling_loc[:, idx].contiguous(),
                                p.weights[:, idx].contiguous(),
                                grad_out[:, idx].contiguous(), need_feat=False)
    return gl, gw
