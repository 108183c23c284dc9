"""PyTorch-facing entry points of the MSDA library.

PyTorch supplies device memory and the current HIP stream; the computation is
the library's (libmsda.so, via ctypes). The operator is multi-scale deformable
aggregation (paper Sec. 3.1 / Sec. 3.2, accelerated in Sec. 5.3):

    out[b, a, :] = sum over keypoints p, cameras n, levels l of
                   weights[b, a, p, n, l, group] * bilinear(feat region (n, l), loc[b, a, p, n])

Layouts are those of include/msda.h. ``Layout`` carries the per-(camera,
level) geometry both on the device (read by the kernels) and on the host
(validated by the library without a device read).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib

_DTYPES = {torch.float32: _lib.MSDA_F32, torch.bfloat16: _lib.MSDA_BF16, torch.float16: _lib.MSDA_F16,
           torch.float8_e4m3fn: _lib.MSDA_FP8_E4M3, torch.uint8: _lib.MSDA_FP8_E4M3}


class Layout:
    """Geometry of the feature rows: spatial_shapes [Ncam, L, 2] (H, W) and
    level_start_index [Ncam, L], kept on the host and on `device`."""

    def __init__(self, spatial_shapes, level_start_index, device="cuda"):
        hs = torch.as_tensor(spatial_shapes).detach().to("cpu", torch.int32).contiguous()
        hl = torch.as_tensor(level_start_index).detach().to("cpu", torch.int32).contiguous()
        if hs.dim() != 3 or hs.shape[2] != 2 or hl.shape != hs.shape[:2]:
            raise ValueError(f"bad geometry shapes {tuple(hs.shape)} / {tuple(hl.shape)}")
        self.host_shapes = hs.numpy().copy()
        self.host_starts = hl.numpy().copy()
        self.shapes = hs.to(device)
        self.starts = hl.to(device)
        self.num_cams, self.num_levels = int(hs.shape[0]), int(hs.shape[1])

    @property
    def rows_needed(self) -> int:
        h, w = self.host_shapes[..., 0].astype(np.int64), self.host_shapes[..., 1].astype(np.int64)
        return int((self.host_starts + h * w).max())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need_cuda_contig(name, t, dtype=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


def _order_code(order) -> int:
    if isinstance(order, str):
        if order not in _lib.ORDERS:
            raise ValueError(f"order must be one of {sorted(_lib.ORDERS)}, got {order!r}")
        return _lib.ORDERS[order]
    return int(order or 0)


def tile_struct(tile: dict, into=None):
    """msda_tile from a dict: waves_per_anchor, chans_per_lane, order
    ("anchor", "view", "auto" or the MSDA_ORDER_* code), scatter."""
    t = into if into is not None else _lib.MsdaTile()
    t.waves_per_anchor = int(tile.get("waves_per_anchor", 0))
    t.chans_per_lane = int(tile.get("chans_per_lane", 0))
    t.order = _order_code(tile.get("order", 0))
    t.scatter = int(tile.get("scatter", 0))
    return t


def make_desc(feat: torch.Tensor, layout: Layout, sampling_loc: torch.Tensor,
              weights: torch.Tensor, level_scale: Optional[torch.Tensor] = None,
              deterministic: bool = False, tile: Optional[dict] = None, logits: bool = False):
    """Build the msda_desc for these tensors (shapes are checked here and,
    authoritatively, by the library)."""
    if feat.dim() != 3 or sampling_loc.dim() != 5 or weights.dim() != 6:
        raise ValueError("feat [B,R,C], sampling_loc [B,A,P,Ncam,2], weights [B,A,P,Ncam,L,G]")
    B, R, C = feat.shape
    _, A, P, N, two = sampling_loc.shape
    if two != 2 or sampling_loc.shape[0] != B or N != layout.num_cams:
        raise ValueError(f"sampling_loc shape {tuple(sampling_loc.shape)} does not match")
    if weights.shape[:5] != (B, A, P, N, layout.num_levels):
        raise ValueError(f"weights shape {tuple(weights.shape)} does not match")
    if feat.dtype not in _DTYPES:
        raise ValueError(f"unsupported feat dtype {feat.dtype}")
    d = _lib.MsdaDesc()
    d.batch, d.num_cams, d.num_levels = B, N, layout.num_levels
    d.num_anchors, d.num_points, d.channels = A, P, C
    d.groups = weights.shape[5]
    d.feat_dtype = _DTYPES[feat.dtype]
    d.rows = R
    d.host_spatial_shapes = layout.host_shapes.ctypes.data
    d.host_level_start_index = layout.host_starts.ctypes.data
    d.level_scale = level_scale.data_ptr() if level_scale is not None else None
    d.flags = ((_lib.MSDA_DETERMINISTIC if deterministic else 0) |
               (_lib.MSDA_WEIGHT_LOGITS if logits else 0) |
               (_lib.MSDA_WEIGHTS_BF16 if weights.dtype == torch.bfloat16 else 0))
    keep = [layout]
    if tile:
        t = tile_struct(tile)
        keep.append(t)
        d.tile = ctypes.pointer(t)
    d._keep = keep        # host arrays must outlive the call
    return d


def _need_weights(weights):
    _need_cuda_contig("weights", weights)
    if weights.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError(f"weights must be float32 or bfloat16, got {weights.dtype}")


def _resolve_tile(tile, which, feat, sampling_loc, weights):
    """tile="auto": the autotuner's cached shape for this workload (or the
    library's own choice when nothing is cached)."""
    if tile != "auto":
        return tile
    from . import autotune
    B, _, C = feat.shape
    A, P, N = sampling_loc.shape[1], sampling_loc.shape[2], sampling_loc.shape[3]
    entry = autotune.lookup(autotune.shape_key(feat.dtype, C, weights.shape[5], weights.shape[4],
                                               P, N, A, B, "single"))
    return entry.get(which) if entry else None


def _workspace(nbytes: int, workspace: Optional[torch.Tensor], device):
    """(pointer, usable bytes) of a 256-byte aligned workspace of at least
    nbytes: the caller's tensor if large enough, else a new one."""
    if not nbytes:
        return None, 0, workspace

    def usable(t):
        base = t.data_ptr()
        aligned = (base + 255) // 256 * 256
        return aligned, t.numel() * t.element_size() - (aligned - base)

    if workspace is None or usable(workspace)[1] < nbytes:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    aligned, n = usable(workspace)
    return ctypes.c_void_p(aligned), n, workspace


def forward_workspace_bytes(feat, layout, sampling_loc, weights, tile=None,
                            logits=False) -> int:
    d = make_desc(feat, layout, sampling_loc, weights, tile=tile, logits=logits)
    return int(_lib.load().msda_forward_workspace_size(ctypes.byref(d)))


def forward(feat, layout: Layout, sampling_loc, weights, level_scale=None, tile=None,
            out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
            stream=None, logits: bool = False) -> torch.Tensor:
    """out [B, A, C] FP32 = MSDA(feat, loc, weights) on the current stream.
    tile: None (the library's choice), a dict of msda_tile fields, or "auto".
    workspace: optional uint8 device tensor for the view-order forward (one
    is allocated when needed and not given). weights: FP32 or BF16; logits:
    they are logits and the per-group softmax over (keypoint, camera, level)
    is applied inside."""
    lib = _lib.load()
    tile = _resolve_tile(tile, "forward", feat, sampling_loc, weights)
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    if level_scale is not None:
        _need_cuda_contig("level_scale", level_scale, torch.float32)
    d = make_desc(feat, layout, sampling_loc, weights, level_scale, tile=tile, logits=logits)
    if out is None:
        out = torch.empty(d.batch, d.num_anchors, d.channels, device=feat.device,
                          dtype=torch.float32)
    ws_ptr, ws_len, workspace = _workspace(int(lib.msda_forward_workspace_size(ctypes.byref(d))),
                                           workspace, feat.device)
    _lib.check(lib.msda_forward_ws(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                   _ptr(sampling_loc), _ptr(weights), _ptr(out), ws_ptr, ws_len,
                                   ctypes.byref(d), _stream(stream)))
    return out


def forward_noalloc(feat, layout: Layout, sampling_loc, weights, out: torch.Tensor,
                    level_scale=None, tile=None, stream=None, logits: bool = False
                    ) -> torch.Tensor:
    """forward() through msda_forward_noalloc: no workspace; the library's
    fixed per-GPU scratch array holds the view order's partial sums. `out`
    [B, A, C] FP32 is given by the caller (nothing is allocated here)."""
    lib = _lib.load()
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    _need_cuda_contig("out", out, torch.float32)
    if level_scale is not None:
        _need_cuda_contig("level_scale", level_scale, torch.float32)
    d = make_desc(feat, layout, sampling_loc, weights, level_scale, tile=tile, logits=logits)
    if tuple(out.shape) != (d.batch, d.num_anchors, d.channels):
        raise ValueError(f"out must be [{d.batch}, {d.num_anchors}, {d.channels}]")
    _lib.check(lib.msda_forward_noalloc(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                        _ptr(sampling_loc), _ptr(weights), _ptr(out),
                                        ctypes.byref(d), _stream(stream)))
    return out


def backward_workspace_bytes(feat, layout, sampling_loc, weights, deterministic=False,
                             tile=None, logits=False) -> int:
    d = make_desc(feat, layout, sampling_loc, weights, deterministic=deterministic, tile=tile,
                  logits=logits)
    return int(_lib.load().msda_backward_workspace_size(ctypes.byref(d)))


def backward(feat, layout: Layout, sampling_loc, weights, grad_out,
             need_feat=True, need_loc=True, need_w=True, deterministic=False, tile=None,
             workspace: Optional[torch.Tensor] = None, level_scale=None, stream=None,
             logits: bool = False
             ) -> Tuple[Optional[torch.Tensor], Optional[torch.Tensor], Optional[torch.Tensor]]:
    """(grad_feat, grad_sampling_loc, grad_weights); an unrequested one is None.
    grad_weights is FP32 (with logits=True: the gradient of the logits)."""
    lib = _lib.load()
    tile = _resolve_tile(tile, "backward", feat, sampling_loc, weights)
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    _need_cuda_contig("grad_out", grad_out, torch.float32)
    d = make_desc(feat, layout, sampling_loc, weights, level_scale, deterministic=deterministic,
                  tile=tile, logits=logits)
    gf = torch.empty_like(feat) if need_feat else None
    gl = torch.empty_like(sampling_loc) if need_loc else None
    gw = torch.empty(weights.shape, dtype=torch.float32, device=weights.device) if need_w else None
    weight_flags = logits or weights.dtype == torch.bfloat16
    ws_bytes = (int(lib.msda_backward_workspace_size(ctypes.byref(d)))
                if need_feat or weight_flags else 0)
    ws_ptr, ws_len, workspace = _workspace(ws_bytes, workspace, feat.device)
    _lib.check(lib.msda_backward(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                 _ptr(sampling_loc), _ptr(weights), _ptr(grad_out), _ptr(gf),
                                 _ptr(gl), _ptr(gw), ws_ptr, ws_len, ctypes.byref(d),
                                 _stream(stream)))
    return gf, gl, gw


def project_keypoints(anchors, keypoints, projection, image_hw, dt: float, stream=None):
    """Keypoint projection with motion compensation on the device:
    (sampling_loc [B, A, P, N, 2] FP32, visible [B, A, N] uint8). anchors
    [B, A, 10], keypoints [B, A, P, 3], projection [B, N, 3, 4] FP32 and
    image_hw [N, 2] int32, all on the device."""
    lib = _lib.load()
    _need_cuda_contig("anchors", anchors, torch.float32)
    _need_cuda_contig("keypoints", keypoints, torch.float32)
    _need_cuda_contig("projection", projection, torch.float32)
    _need_cuda_contig("image_hw", image_hw, torch.int32)
    B, A, P, three = keypoints.shape
    N = projection.shape[1]
    if three != 3 or anchors.shape != (B, A, 10) or projection.shape != (B, N, 3, 4) or \
            image_hw.shape != (N, 2):
        raise ValueError("anchors [B,A,10], keypoints [B,A,P,3], projection [B,N,3,4], "
                         "image_hw [N,2]")
    loc = torch.empty(B, A, P, N, 2, dtype=torch.float32, device=anchors.device)
    vis = torch.empty(B, A, N, dtype=torch.uint8, device=anchors.device)
    d = _lib.MsdaProjDesc(B, A, P, N, float(dt))
    _lib.check(lib.msda_project_keypoints(_ptr(anchors), _ptr(keypoints), _ptr(projection),
                                          _ptr(image_hw), _ptr(loc), _ptr(vis), ctypes.byref(d),
                                          _stream(stream)))
    return loc, vis


def _need_visible(visible, sampling_loc):
    _need_cuda_contig("visible", visible, torch.uint8)
    B, A, _, N, _ = sampling_loc.shape
    if visible.shape != (B, A, N):
        raise ValueError(f"visible must be [B, A, Ncam] = {(B, A, N)}, got {tuple(visible.shape)}")


def forward_visible(feat, layout: Layout, sampling_loc, weights, visible, level_scale=None,
                    tile=None, out: Optional[torch.Tensor] = None,
                    workspace: Optional[torch.Tensor] = None, stream=None,
                    logits: bool = False) -> torch.Tensor:
    """out [B, A, C] = MSDA over the visible (anchor, camera) pairs only
    (weights FP32 or BF16; logits: per-group softmax logits)."""
    lib = _lib.load()
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    _need_visible(visible, sampling_loc)
    d = make_desc(feat, layout, sampling_loc, weights, level_scale, tile=tile, logits=logits)
    if out is None:
        out = torch.empty(d.batch, d.num_anchors, d.channels, device=feat.device,
                          dtype=torch.float32)
    ws_ptr, ws_len, workspace = _workspace(
        int(lib.msda_forward_visible_workspace_size(ctypes.byref(d))), workspace, feat.device)
    _lib.check(lib.msda_forward_visible(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                        _ptr(sampling_loc), _ptr(weights), _ptr(visible),
                                        _ptr(out), ws_ptr, ws_len, ctypes.byref(d),
                                        _stream(stream)))
    return out


def backward_visible(feat, layout: Layout, sampling_loc, weights, visible, grad_out,
                     need_feat=True, need_loc=True, need_w=True, tile=None,
                     workspace: Optional[torch.Tensor] = None, stream=None,
                     logits: bool = False):
    """(grad_feat, grad_sampling_loc, grad_weights) of the visible-view form;
    the gradients of invisible pairs are zero (with logits, grad_weights is
    the logits' gradient, which reaches invisible entries through the
    softmax's normalisation)."""
    lib = _lib.load()
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    _need_cuda_contig("grad_out", grad_out, torch.float32)
    _need_visible(visible, sampling_loc)
    d = make_desc(feat, layout, sampling_loc, weights, tile=tile, logits=logits)
    gf = torch.empty_like(feat) if need_feat else None
    gl = torch.empty_like(sampling_loc) if need_loc else None
    gw = torch.empty(weights.shape, dtype=torch.float32, device=weights.device) if need_w else None
    ws_ptr, ws_len, workspace = _workspace(
        int(lib.msda_backward_visible_workspace_size(ctypes.byref(d))), workspace, feat.device)
    _lib.check(lib.msda_backward_visible(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                         _ptr(sampling_loc), _ptr(weights), _ptr(visible),
                                         _ptr(grad_out), _ptr(gf), _ptr(gl), _ptr(gw), ws_ptr,
                                         ws_len, ctypes.byref(d), _stream(stream)))
    return gf, gl, gw


def _need_scores(view_score, visible):
    _need_cuda_contig("view_score", view_score, torch.float32)
    if view_score.shape != visible.shape:
        raise ValueError(f"view_score must be [B, A, Ncam] = {tuple(visible.shape)}, "
                         f"got {tuple(view_score.shape)}")


def forward_fused(feat, layout: Layout, sampling_loc, weights, visible, view_score,
                  level_scale=None, tile=None, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None,
                  logits: bool = False) -> torch.Tensor:
    """out [B, A, C]: the visible views' features weighted by view_score over
    the visible cameras' score sum (visibility-weighted fusion, Eq. 2)."""
    lib = _lib.load()
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    _need_visible(visible, sampling_loc)
    _need_scores(view_score, visible)
    d = make_desc(feat, layout, sampling_loc, weights, level_scale, tile=tile, logits=logits)
    if out is None:
        out = torch.empty(d.batch, d.num_anchors, d.channels, device=feat.device,
                          dtype=torch.float32)
    ws_ptr, ws_len, workspace = _workspace(
        int(lib.msda_forward_fused_workspace_size(ctypes.byref(d))), workspace, feat.device)
    _lib.check(lib.msda_forward_fused(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                      _ptr(sampling_loc), _ptr(weights), _ptr(visible),
                                      _ptr(view_score), _ptr(out), ws_ptr, ws_len,
                                      ctypes.byref(d), _stream(stream)))
    return out


def backward_fused(feat, layout: Layout, sampling_loc, weights, visible, view_score, out,
                   grad_out, need_feat=True, need_loc=True, need_w=True, need_score=True,
                   tile=None, workspace: Optional[torch.Tensor] = None, stream=None,
                   logits: bool = False):
    """(grad_feat, grad_sampling_loc, grad_weights, grad_score) of
    forward_fused; out is forward_fused's result (needed for grad_score)."""
    lib = _lib.load()
    _need_cuda_contig("feat", feat)
    _need_cuda_contig("sampling_loc", sampling_loc, torch.float32)
    _need_weights(weights)
    _need_cuda_contig("grad_out", grad_out, torch.float32)
    _need_visible(visible, sampling_loc)
    _need_scores(view_score, visible)
    if need_score:
        _need_cuda_contig("out", out, torch.float32)
        if out.shape != grad_out.shape:
            raise ValueError(f"out must match grad_out {tuple(grad_out.shape)}, "
                             f"got {tuple(out.shape)}")
    d = make_desc(feat, layout, sampling_loc, weights, tile=tile, logits=logits)
    gf = torch.empty_like(feat) if need_feat else None
    gl = torch.empty_like(sampling_loc) if need_loc else None
    gw = torch.empty(weights.shape, dtype=torch.float32, device=weights.device) if need_w else None
    gs = torch.empty_like(view_score) if need_score else None
    ws_ptr, ws_len, workspace = _workspace(
        int(lib.msda_backward_fused_workspace_size(ctypes.byref(d))), workspace, feat.device)
    _lib.check(lib.msda_backward_fused(_ptr(feat), _ptr(layout.shapes), _ptr(layout.starts),
                                       _ptr(sampling_loc), _ptr(weights), _ptr(visible),
                                       _ptr(view_score), _ptr(out if need_score else None),
                                       _ptr(grad_out), _ptr(gf), _ptr(gl), _ptr(gw), _ptr(gs),
                                       ws_ptr, ws_len, ctypes.byref(d), _stream(stream)))
    return gf, gl, gw, gs


def quantize_fp8(feat_f32: torch.Tensor, layout: Layout, stream=None):
    """Per-level FP8 e4m3 quantisation on the device: (codes uint8 [B,R,C],
    level_scale float32 [L]) with scale_l = amax_l / 448."""
    lib = _lib.load()
    _need_cuda_contig("feat", feat_f32, torch.float32)
    B, R, C = feat_f32.shape
    d = _lib.MsdaDesc()
    d.batch, d.num_cams, d.num_levels = B, layout.num_cams, layout.num_levels
    d.num_anchors, d.num_points, d.channels, d.groups = 0, 1, C, 1
    d.feat_dtype, d.rows = _lib.MSDA_F32, R
    d.host_spatial_shapes = layout.host_shapes.ctypes.data
    d.host_level_start_index = layout.host_starts.ctypes.data
    codes = torch.empty(B, R, C, dtype=torch.uint8, device=feat_f32.device)
    scales = torch.empty(layout.num_levels, dtype=torch.float32, device=feat_f32.device)
    ws = torch.empty(max(16, int(lib.msda_quantize_workspace_size(ctypes.byref(d)))),
                     dtype=torch.uint8, device=feat_f32.device)
    _lib.check(lib.msda_quantize_fp8(_ptr(feat_f32), _ptr(layout.shapes), _ptr(layout.starts),
                                     _ptr(codes), _ptr(scales), _ptr(ws), ws.numel(),
                                     ctypes.byref(d), _stream(stream)))
    return codes, scales


def sort_keys(keys: torch.Tensor, max_key: int, stream=None):
    """Stable sort of uint32 keys (an int32 or uint32 device tensor, values in
    [0, max_key]) with the backward's record sort: (order int32 [n],
    seg int32 [max_key + 1]) where order lists the indices by key, equal keys
    in index order, and seg[r] is the first sorted position whose key >= r."""
    lib = _lib.load()
    if keys.dtype not in (torch.int32, torch.uint32) or not keys.is_cuda or keys.dim() != 1:
        raise ValueError("keys must be a 1-D int32/uint32 device tensor")
    keys = keys.contiguous()
    n = keys.numel()
    order = torch.empty(n, dtype=torch.int32, device=keys.device)
    seg = torch.empty(max_key + 1, dtype=torch.int32, device=keys.device)
    ws = torch.empty(max(256, int(lib.msda_sort_workspace_size(n, max_key))), dtype=torch.uint8,
                     device=keys.device)
    _lib.check(lib.msda_sort_keys(_ptr(keys) if n else None, n, max_key,
                                  _ptr(order) if n else None, _ptr(seg), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return order, seg


def stream_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """Plain streaming copy kernel (the achievable-bandwidth reference)."""
    lib = _lib.load()
    n = src.numel() * src.element_size()
    _lib.check(lib.msda_stream_copy(_ptr(dst), _ptr(src), n, _stream(stream)))


class MSDAFunction(torch.autograd.Function):
    """Differentiable MSDA: forward and backward are the library's kernels.
    No gradient flows to the geometry or to the FP8 level scales. With
    logits=True the weights argument holds logits (softmax applied inside)
    and receives their gradient; a BF16 weights tensor gets an FP32
    gradient cast to BF16 by autograd's dtype rule."""

    @staticmethod
    def forward(ctx, feat, sampling_loc, weights, layout, level_scale, deterministic, tile,
                logits):
        out = forward(feat, layout, sampling_loc, weights, level_scale=level_scale, tile=tile,
                      logits=logits)
        ctx.save_for_backward(feat, sampling_loc, weights)
        ctx.layout, ctx.deterministic, ctx.tile = layout, deterministic, tile
        ctx.level_scale, ctx.logits = level_scale, logits
        return out

    @staticmethod
    def backward(ctx, grad_out):
        feat, loc, w = ctx.saved_tensors
        nf, nl, nw = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gf = gl = gw = None
        if nf or nl or nw:
            gf, gl, gw = backward(feat, ctx.layout, loc, w, grad_out.contiguous(),
                                  need_feat=nf, need_loc=nl, need_w=nw,
                                  deterministic=ctx.deterministic, tile=ctx.tile,
                                  level_scale=ctx.level_scale, logits=ctx.logits)
            if gw is not None and gw.dtype != w.dtype:
                gw = gw.to(w.dtype)
        return gf, gl, gw, None, None, None, None, None


def msda(feat, layout: Layout, sampling_loc, weights, level_scale=None, deterministic=False,
         tile=None, logits=False):
    """Autograd-aware MSDA (logits=True: weights are per-group softmax logits)."""
    return MSDAFunction.apply(feat, sampling_loc, weights, layout, level_scale, deterministic,
                              tile, logits)


class SceneBatch:
    """Uneven scenes processed together: the batched form of MSDA.

    Each scene has its own cameras, feature geometry and anchors; levels,
    keypoints, channels, groups and the feature dtype are shared. The batch
    owns every output and gradient buffer and a device copy of the scene
    table, built once here, so forward() / backward() allocate nothing and
    can be captured in a HIP graph (torch.cuda.graph). Write each scene's
    upstream gradient into ``grad_out[s]`` before backward().

    scenes: list of (feat [R, C], Layout, sampling_loc [A, P, Ncam, 2],
    weights [A, P, Ncam, L, G]) on the device; weights FP32 or BF16 (the same
    in every scene). logits: the weights are per-group logits, turned into
    the softmax over each anchor's (keypoint, camera, level) entries inside,
    and grad_w is the logits' gradient (FP32).
    """

    def __init__(self, scenes, level_scale=None, need_feat=True, need_loc=True, need_w=True,
                 tile=None, deterministic=False, logits: bool = False):
        lib = _lib.load()
        if not scenes:
            raise ValueError("empty batch")
        feat0, lay0, loc0, w0 = scenes[0]
        self.device = feat0.device
        self.C = feat0.shape[-1]
        self.L, self.G = w0.shape[-2], w0.shape[-1]
        self.P = loc0.shape[1]
        self.dtype = feat0.dtype
        self.w_dtype = w0.dtype
        self.scenes = scenes
        self.level_scale = level_scale
        self.out, self.grad_out, self.grad_feat, self.grad_loc, self.grad_w = [], [], [], [], []
        n = len(scenes)
        host = (_lib.MsdaScene * n)()
        self._host_shapes = (ctypes.c_void_p * n)()
        self._host_starts = (ctypes.c_void_p * n)()
        for s, (feat, layout, loc, w) in enumerate(scenes):
            for name, t in (("feat", feat), ("sampling_loc", loc), ("weights", w)):
                _need_cuda_contig(f"scene {s} {name}", t)
            if feat.dim() != 2 or loc.dim() != 4 or w.dim() != 5:
                raise ValueError("scene tensors: feat [R,C], loc [A,P,Ncam,2], w [A,P,Ncam,L,G]")
            if feat.dtype != self.dtype or feat.shape[1] != self.C:
                raise ValueError(f"scene {s}: feat dtype / channels differ from scene 0")
            if w.dtype != self.w_dtype or w.dtype not in (torch.float32, torch.bfloat16):
                raise ValueError(f"scene {s}: weights must be FP32 or BF16, as scene 0's")
            A = loc.shape[0]
            # keypoints, levels and groups are shared by the batch (the kernels
            # read every scene's locations and weights with scene 0's sizes)
            if loc.shape != (A, self.P, layout.num_cams, 2):
                raise ValueError(f"scene {s}: sampling_loc {tuple(loc.shape)} is not "
                                 f"[A, P={self.P}, Ncam={layout.num_cams}, 2]")
            if w.shape != (A, self.P, layout.num_cams, self.L, self.G):
                raise ValueError(f"scene {s}: weights {tuple(w.shape)} is not "
                                 f"[A, P={self.P}, Ncam={layout.num_cams}, L={self.L}, G={self.G}]")
            out = torch.empty(A, self.C, device=self.device, dtype=torch.float32)
            go = torch.zeros(A, self.C, device=self.device, dtype=torch.float32)
            gf = torch.empty_like(feat) if need_feat else None
            gl = torch.empty_like(loc) if need_loc else None
            gw = torch.empty(w.shape, dtype=torch.float32, device=w.device) if need_w else None
            self.out.append(out)
            self.grad_out.append(go)
            self.grad_feat.append(gf)
            self.grad_loc.append(gl)
            self.grad_w.append(gw)
            h = host[s]
            h.feat, h.spatial_shapes = feat.data_ptr(), layout.shapes.data_ptr()
            h.level_start_index = layout.starts.data_ptr()
            h.sampling_loc, h.weights = loc.data_ptr(), w.data_ptr()
            h.out, h.grad_out = out.data_ptr(), go.data_ptr()
            h.grad_feat = gf.data_ptr() if gf is not None else None
            h.grad_sampling_loc = gl.data_ptr() if gl is not None else None
            h.grad_weights = gw.data_ptr() if gw is not None else None
            h.rows, h.num_cams, h.num_anchors = feat.shape[0], layout.num_cams, A
            if layout.num_levels != self.L:
                raise ValueError(f"scene {s}: {layout.num_levels} levels, scene 0 has {self.L}")
            self._host_shapes[s] = layout.host_shapes.ctypes.data
            self._host_starts[s] = layout.host_starts.ctypes.data
        self._host = host
        raw = bytes(host)
        self._dev_table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        b = _lib.MsdaBatch()
        b.num_scenes, b.num_levels, b.num_points = n, self.L, self.P
        b.channels, b.groups, b.feat_dtype = self.C, self.G, _DTYPES[self.dtype]
        b.scenes = self._dev_table.data_ptr()
        b.host_scenes = ctypes.cast(host, ctypes.POINTER(_lib.MsdaScene))
        b.host_spatial_shapes = ctypes.cast(self._host_shapes, ctypes.POINTER(ctypes.c_void_p))
        b.host_level_start_index = ctypes.cast(self._host_starts, ctypes.POINTER(ctypes.c_void_p))
        b.level_scale = level_scale.data_ptr() if level_scale is not None else None
        b.flags = ((_lib.MSDA_DETERMINISTIC if deterministic else 0) |
                   (_lib.MSDA_WEIGHT_LOGITS if logits else 0) |
                   (_lib.MSDA_WEIGHTS_BF16 if self.w_dtype == torch.bfloat16 else 0))
        self._batch = b
        self._tile = _lib.MsdaTile()
        if tile == "auto":
            from . import autotune
            cams = max(layout.num_cams for _, layout, _, _ in scenes)
            anchors = sum(loc.shape[0] for _, _, loc, _ in scenes)
            entry = autotune.lookup(autotune.shape_key(self.dtype, self.C, self.G, self.L, self.P,
                                                       cams, anchors, 1, "batch"))
            tile = entry.get("tile") if entry else None
        self.set_tile(tile)
        fwd_ws = int(lib.msda_batched_workspace_size(ctypes.byref(b), 0))
        bwd_ws = int(lib.msda_batched_workspace_size(ctypes.byref(b), 1))
        # the size query returns 0 for an invalid batch: a call without a
        # workspace then reports why (validation comes first)
        if fwd_ws == 0:
            _lib.check(lib.msda_forward_batched(ctypes.byref(b), None, 0, None))
        if bwd_ws == 0:
            _lib.check(lib.msda_backward_batched(ctypes.byref(b), None, 0, None))
        self._ws = torch.empty(max(fwd_ws, bwd_ws) + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ws_len = self._ws.numel() - (self._ws_ptr - base)

    def set_tile(self, tile: Optional[dict]):
        """Launch shape of later calls: None for the library's choice."""
        if tile:
            tile_struct(tile, self._tile)
            self._batch.tile = ctypes.pointer(self._tile)
        else:
            self._batch.tile = None
        self.tile = dict(tile) if tile else None

    @property
    def samples(self) -> int:
        return sum(loc.shape[0] * loc.shape[1] * loc.shape[2] * self.L
                   for _, _, loc, _ in self.scenes)

    def forward(self, stream=None):
        lib = _lib.load()
        _lib.check(lib.msda_forward_batched(ctypes.byref(self._batch), ctypes.c_void_p(self._ws_ptr),
                                            self._ws_len, _stream(stream)))
        return self.out

    def backward(self, stream=None):
        lib = _lib.load()
        _lib.check(lib.msda_backward_batched(ctypes.byref(self._batch),
                                             ctypes.c_void_p(self._ws_ptr), self._ws_len,
                                             _stream(stream)))
        return self.grad_feat, self.grad_loc, self.grad_w
