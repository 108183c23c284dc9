"""The C ABI: the library loads, exports every symbol include/msda.h declares,
and rejects bad arguments on the host before anything is launched. These
tests pass fake device addresses and only exercise failure paths (plus the
empty A=0 case, which launches nothing), so they run without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2601_10819_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x7f0000000000           # 16-byte aligned stand-in for a device address


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "msda.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msda_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert "msda_forward" in syms and "msda_backward" in syms
    for s in syms:
        assert hasattr(lib, s), f"libmsda.so does not export {s}"
    assert set(syms) == set(_lib.EXPORTS)
    assert lib.msda_abi_version() == _lib.ABI_VERSION


class Geo:
    def __init__(self, ncam=2, levels=((8, 12), (4, 6)), rows=None):
        shapes, starts, r = [], [], 0
        for _ in range(ncam):
            for h, w in levels:
                shapes.append((h, w))
                starts.append(r)
                r += h * w
        self.shapes = np.array(shapes, dtype=np.int32).reshape(ncam, len(levels), 2)
        self.starts = np.array(starts, dtype=np.int32).reshape(ncam, len(levels))
        self.rows = r if rows is None else rows


def desc(geo, B=1, A=4, P=3, C=32, G=4, dtype=_lib.MSDA_F32, scale=None, flags=0, tile=None):
    d = _lib.MsdaDesc()
    d.batch, d.num_cams, d.num_levels = B, geo.shapes.shape[0], geo.shapes.shape[1]
    d.num_anchors, d.num_points, d.channels, d.groups = A, P, C, G
    d.feat_dtype, d.rows = dtype, geo.rows
    d.host_spatial_shapes = geo.shapes.ctypes.data
    d.host_level_start_index = geo.starts.ctypes.data
    d.level_scale = scale
    d.flags = flags
    if tile is not None:
        d._t = _lib.MsdaTile(*tile)
        d.tile = ctypes.pointer(d._t)
    d._geo = geo
    return d


def fwd(lib, d, feat=FAKE, out=FAKE + 4096):
    return lib.msda_forward(feat, FAKE, FAKE, FAKE, FAKE, out, ctypes.byref(d), None)


def bwd(lib, d, grad_feat=FAKE + 8192, ws=None, ws_bytes=0, feat=FAKE):
    return lib.msda_backward(feat, FAKE, FAKE, FAKE, FAKE, FAKE, grad_feat, FAKE, FAKE, ws,
                             ws_bytes, ctypes.byref(d), None)


def expect(lib, status, want, needle=None):
    assert status == want, (status, lib.msda_last_error())
    msg = lib.msda_last_error().decode()
    assert msg, "a failure must leave a message"
    if needle:
        assert needle in msg, msg


INV, UNS, WS = _lib.MSDA_ERR_INVALID_ARGUMENT, _lib.MSDA_ERR_UNSUPPORTED, _lib.MSDA_ERR_WORKSPACE


def test_null_desc_and_pointers(lib):
    expect(lib, lib.msda_forward(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None, None), INV, "desc")
    d = desc(Geo())
    expect(lib, fwd(lib, d, feat=None), INV, "NULL")
    expect(lib, fwd(lib, d, out=None), INV, "NULL")
    d.host_spatial_shapes = None
    expect(lib, fwd(lib, d), INV, "host mirrors")


@pytest.mark.parametrize("field,value", [("batch", 0), ("num_cams", 0), ("num_levels", 0),
                                         ("num_anchors", -1), ("num_points", 0), ("channels", 0),
                                         ("groups", 0), ("rows", 0), ("batch", -3)])
def test_nonpositive_sizes(lib, field, value):
    d = desc(Geo())
    setattr(d, field, value)
    expect(lib, fwd(lib, d), INV)


def test_channels_not_divisible_by_groups(lib):
    expect(lib, fwd(lib, desc(Geo(), C=30, G=4)), INV, "divisible")


def test_region_outside_rows(lib):
    g = Geo()
    g.rows -= 1
    expect(lib, fwd(lib, desc(g)), INV, "outside")
    g = Geo()
    g.starts[1, 0] = -5
    expect(lib, fwd(lib, desc(g)), INV, "outside")


def test_bad_level_shape(lib):
    g = Geo()
    g.shapes[0, 1, 1] = 0
    expect(lib, fwd(lib, desc(g)), INV, "H=")
    g = Geo()
    g.shapes[1, 0, 0] = -2
    expect(lib, fwd(lib, desc(g)), INV)


def test_unknown_dtype_and_fp8_scale(lib):
    expect(lib, fwd(lib, desc(Geo(), dtype=7)), INV, "dtype")
    expect(lib, fwd(lib, desc(Geo(), dtype=_lib.MSDA_FP8_E4M3, C=64)), INV, "level_scale")


def test_unsupported_requests(lib):
    expect(lib, fwd(lib, desc(Geo(), C=96, G=3)), UNS, "lane layout")
    expect(lib, fwd(lib, desc(Geo(levels=tuple((2, 2) for _ in range(9))))), UNS, "levels")
    expect(lib, fwd(lib, desc(Geo()), feat=FAKE + 4), UNS, "aligned")
    expect(lib, fwd(lib, desc(Geo(), tile=(3, 0, 0, 0))), UNS, "waves_per_anchor")
    expect(lib, fwd(lib, desc(Geo(), tile=(0, 16, 0, 0))), UNS, "chans_per_lane")
    expect(lib, fwd(lib, desc(Geo(), tile=(0, 0, 5, 0))), UNS, "order")
    # one batch item beyond 4 GiB - 8 KiB of features (4096 x 4096 x 64 FP32)
    g = Geo(ncam=1, levels=((4096, 4096),))
    expect(lib, fwd(lib, desc(g, C=64, G=4)), UNS, "bytes")
    # 2 GiB < one batch item <= 4 GiB - 8 KiB is accepted (validation only here)
    g = Geo(ncam=2, levels=((1024, 2000),))
    assert fwd(lib, desc(g, C=256, G=8, A=0)) == _lib.MSDA_OK
    # a feature row above 4 KiB (its offset plus the out-of-level marker
    # would pass 2^32; the lane layouts stop at 1 KiB rows anyway)
    expect(lib, fwd(lib, desc(Geo(), C=2048, G=8)), UNS, "row")


def test_backward_validation(lib):
    d = desc(Geo(), dtype=_lib.MSDA_FP8_E4M3, C=64, scale=FAKE)
    expect(lib, bwd(lib, d), UNS, "FP8")
    # sorted grad_feat (the default): keys, values (twice each), fractions
    # (8 bytes) per sample and one offset per bilinear cell
    d = desc(Geo(), dtype=_lib.MSDA_BF16, C=64)
    need = lib.msda_backward_workspace_size(ctypes.byref(d))
    nsamp = 1 * 4 * 3 * 2 * 2
    ncells = 2 * ((8 + 1) * (12 + 1) + (4 + 1) * (6 + 1))
    assert need >= 4 * 4 * nsamp + 8 * nsamp + 4 * (ncells + 1)
    expect(lib, bwd(lib, d), WS, "workspace")
    expect(lib, bwd(lib, d, ws=FAKE + (1 << 20), ws_bytes=need - 4), WS)
    expect(lib, bwd(lib, d, ws=(FAKE + (1 << 20)) + 8, ws_bytes=need + 64), WS, "aligned")
    # no grad_feat: no workspace needed, so none is checked
    # atomic grad_feat: FP32 needs none, BF16 an FP32 accumulator
    d = desc(Geo(), tile=(0, 0, 0, _lib.MSDA_SCATTER_ATOMIC))
    assert lib.msda_backward_workspace_size(ctypes.byref(d)) == 0
    d = desc(Geo(), dtype=_lib.MSDA_BF16, C=64, tile=(0, 0, 0, _lib.MSDA_SCATTER_ATOMIC))
    assert lib.msda_backward_workspace_size(ctypes.byref(d)) == Geo().rows * 64 * 4
    # deterministic excludes the atomic form; unknown forms are rejected
    d = desc(Geo(), flags=_lib.MSDA_DETERMINISTIC, tile=(0, 0, 0, _lib.MSDA_SCATTER_ATOMIC))
    expect(lib, bwd(lib, d), UNS, "DETERMINISTIC")
    d = desc(Geo(), tile=(0, 0, 0, 7))
    expect(lib, bwd(lib, d, ws=FAKE + (1 << 20), ws_bytes=1 << 30), UNS, "scatter")


def test_kernel_event_hook_validation(lib):
    expect(lib, lib.msda_set_kernel_events(FAKE, 0), INV, "max_kernels")
    assert lib.msda_set_kernel_events(None, 0) == _lib.MSDA_OK
    assert lib.msda_recorded_kernels() == 0
    assert lib.msda_recorded_kernel_name(0) == b""
    expect(lib, lib.msda_set_kernel_event_filter(b"k" * 256), INV, "255")
    assert lib.msda_set_kernel_event_filter(b"radix_scatter") == _lib.MSDA_OK
    assert lib.msda_set_kernel_event_filter(None) == _lib.MSDA_OK


def test_empty_anchor_set_is_ok_without_launch(lib):
    d = desc(Geo(), A=0)
    assert fwd(lib, d) == _lib.MSDA_OK
    assert lib.msda_last_error().decode() == ""


def test_stream_copy_validation(lib):
    expect(lib, lib.msda_stream_copy(None, FAKE, 16, None), INV)
    expect(lib, lib.msda_stream_copy(FAKE, FAKE, 17, None), INV, "aligned")
    expect(lib, lib.msda_stream_copy(FAKE + 4, FAKE, 16, None), INV, "aligned")


def test_quantize_validation(lib):
    d = desc(Geo(), C=64)
    ws = lib.msda_quantize_workspace_size(ctypes.byref(d))
    assert ws == 2 * 2 * 4                     # one word per (camera, level) region
    assert lib.msda_quantize_workspace_size(ctypes.byref(desc(Geo(), B=3, C=64))) == 3 * 2 * 2 * 4
    expect(lib, lib.msda_quantize_fp8(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ws - 4, ctypes.byref(d),
                                      None), WS)
    expect(lib, lib.msda_quantize_fp8(FAKE, FAKE, FAKE, FAKE, FAKE, None, 0, ctypes.byref(d), None),
           WS)
    g = Geo()
    g.rows -= 3
    expect(lib, lib.msda_quantize_fp8(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 64,
                                      ctypes.byref(desc(g, C=64)), None), INV, "outside")


def test_noalloc_refuses_oversize_before_any_hip_call(lib):
    """msda_forward_noalloc checks the workspace it would need against its
    fixed scratch array first, so on a machine without a GPU an input too
    large is refused by size, not by the failed device lookup."""
    expect(lib, lib.msda_forward_noalloc(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None, None), INV)
    d = desc(Geo(ncam=8), A=4200, C=256, G=8, dtype=_lib.MSDA_BF16)
    need = lib.msda_forward_workspace_size(ctypes.byref(d))
    assert need == 8 * 4200 * 256 * 4 > (32 << 20)
    expect(lib, lib.msda_forward_noalloc(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ctypes.byref(d),
                                         None), UNS, "scratch")
    d = desc(Geo(ncam=8), A=4096, C=256, G=8, dtype=_lib.MSDA_BF16)
    assert lib.msda_forward_workspace_size(ctypes.byref(d)) == 32 << 20   # fits exactly


def test_python_binding_fails_loudly_without_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_2601_10819_amd._lib")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            mod.load(str(tmp_path / "nope.so"))
    finally:
        mod._lib = saved


def batch_desc(geos, anchors, grads=(True, True, True)):
    n = len(geos)
    host = (_lib.MsdaScene * n)()
    shp = (ctypes.c_void_p * n)()
    sts = (ctypes.c_void_p * n)()
    for s, (g, a) in enumerate(zip(geos, anchors)):
        h = host[s]
        h.feat = h.spatial_shapes = h.level_start_index = FAKE
        h.sampling_loc = h.weights = h.out = h.grad_out = FAKE
        h.grad_feat = FAKE if grads[0] else None
        h.grad_sampling_loc = FAKE if grads[1] else None
        h.grad_weights = FAKE if grads[2] else None
        h.rows, h.num_cams, h.num_anchors = g.rows, g.shapes.shape[0], a
        shp[s] = g.shapes.ctypes.data
        sts[s] = g.starts.ctypes.data
    b = _lib.MsdaBatch()
    b.num_scenes, b.num_levels, b.num_points, b.channels, b.groups = n, geos[0].shapes.shape[1], 3, 32, 4
    b.feat_dtype = _lib.MSDA_F32
    b.scenes = FAKE
    b.host_scenes = ctypes.cast(host, ctypes.POINTER(_lib.MsdaScene))
    b.host_spatial_shapes = ctypes.cast(shp, ctypes.POINTER(ctypes.c_void_p))
    b.host_level_start_index = ctypes.cast(sts, ctypes.POINTER(ctypes.c_void_p))
    b._keep = (host, shp, sts, geos)
    return b


def test_batched_validation(lib):
    geos = [Geo(ncam=2), Geo(ncam=5, levels=((6, 10), (3, 5)))]
    b = batch_desc(geos, [4, 7])
    fwd_ws = lib.msda_batched_workspace_size(ctypes.byref(b), 0)
    bwd_ws = lib.msda_batched_workspace_size(ctypes.byref(b), 1)
    assert 0 < fwd_ws < bwd_ws
    expect(lib, lib.msda_forward_batched(ctypes.byref(b), None, 0, None), WS, "workspace")
    expect(lib, lib.msda_backward_batched(ctypes.byref(b), FAKE, bwd_ws - 1, None), WS)
    b.num_scenes = 0
    expect(lib, lib.msda_forward_batched(ctypes.byref(b), FAKE, 1 << 30, None), INV, "num_scenes")
    assert lib.msda_batched_workspace_size(ctypes.byref(b), 0) == 0
    # a scene whose regions leave its rows
    bad = Geo(ncam=2)
    bad.rows -= 1
    b = batch_desc([Geo(ncam=2), bad], [4, 4])
    expect(lib, lib.msda_forward_batched(ctypes.byref(b), FAKE, 1 << 30, None), INV, "scene 1")
    # gradients requested by some scenes only
    b = batch_desc(geos, [4, 7])
    b.host_scenes[1].grad_weights = None
    expect(lib, lib.msda_backward_batched(ctypes.byref(b), FAKE, 1 << 30, None), INV, "NULL in all")
    # more (camera, level) regions than the batched tables hold
    big = [Geo(ncam=64, levels=((2, 2),) * 4) for _ in range(17)]
    b = batch_desc(big, [1] * 17)
    expect(lib, lib.msda_forward_batched(ctypes.byref(b), FAKE, 1 << 30, None), UNS, "regions")
    # the batched backward has no atomic form
    b = batch_desc(geos, [4, 7])
    t = _lib.MsdaTile(0, 0, 0, _lib.MSDA_SCATTER_ATOMIC)
    b.tile = ctypes.pointer(t)
    expect(lib, lib.msda_backward_batched(ctypes.byref(b), FAKE, 1 << 30, None), UNS, "sorted")
    # unknown flags are rejected; the weight flags are taken, and grow the
    # workspace by the softmax statistics (and, backward, FP32 weights)
    b = batch_desc(geos, [4, 7])
    b.flags = 1 << 20
    expect(lib, lib.msda_forward_batched(ctypes.byref(b), FAKE, 1 << 30, None), INV, "flags")
    b = batch_desc(geos, [4, 7])
    plain = [lib.msda_batched_workspace_size(ctypes.byref(b), k) for k in (0, 1)]
    b.flags = _lib.MSDA_WEIGHT_LOGITS
    logit = [lib.msda_batched_workspace_size(ctypes.byref(b), k) for k in (0, 1)]
    b.flags = _lib.MSDA_WEIGHTS_BF16
    bf16 = [lib.msda_batched_workspace_size(ctypes.byref(b), k) for k in (0, 1)]
    assert 0 < plain[0] < logit[0] and plain[1] < logit[1], (plain, logit)
    assert bf16[0] == plain[0] and bf16[1] > plain[1], (plain, bf16)
    # an order the batched form does not know
    b = batch_desc(geos, [4, 7])
    t = _lib.MsdaTile(0, 0, 7, 0)
    b.tile = ctypes.pointer(t)
    expect(lib, lib.msda_forward_batched(ctypes.byref(b), FAKE, 1 << 30, None), UNS, "unknown order")
    # the forward's workspace holds the view order's per-slot partial sums
    # (8 x anchors x C FP32) in either order
    b = batch_desc(geos, [4, 7])
    va = lib.msda_batched_workspace_size(ctypes.byref(b), 0)
    t = _lib.MsdaTile(0, 0, _lib.MSDA_ORDER_ANCHOR, 0)
    b.tile = ctypes.pointer(t)
    assert lib.msda_batched_workspace_size(ctypes.byref(b), 0) == va
    assert va >= 8 * 11 * b.channels * 4


def fwd_ws(lib, d, ws=None, ws_bytes=0):
    return lib.msda_forward_ws(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE + 4096, ws, ws_bytes,
                               ctypes.byref(d), None)


def test_view_order_forward_workspace(lib):
    # 2 (batch item, camera) views: the library keeps anchor order, no workspace
    d = desc(Geo(), A=4, C=32)
    assert lib.msda_forward_workspace_size(ctypes.byref(d)) == 0
    # 4 x 2 = 8 views: view order, 8 partial sums per (batch item, anchor)
    d = desc(Geo(), B=4, A=4, C=32)
    need = lib.msda_forward_workspace_size(ctypes.byref(d))
    assert need == 8 * 4 * 4 * 32 * 4
    expect(lib, fwd_ws(lib, d), WS, "workspace")
    expect(lib, fwd_ws(lib, d, ws=FAKE + (1 << 20), ws_bytes=need - 4), WS)
    expect(lib, fwd_ws(lib, d, ws=FAKE + (1 << 20) + 8, ws_bytes=need + 64), WS, "aligned")
    # the plain forward cannot run in view order: asked for explicitly, it says why
    d = desc(Geo(), tile=(0, 0, _lib.MSDA_ORDER_VIEW, 0))
    expect(lib, fwd(lib, d), WS, "msda_forward_ws")
    assert lib.msda_forward_workspace_size(ctypes.byref(d)) == 8 * 1 * 4 * 32 * 4
    # anchor order asked for: no workspace whatever the view count
    d = desc(Geo(), B=4, tile=(0, 0, _lib.MSDA_ORDER_ANCHOR, 0))
    assert lib.msda_forward_workspace_size(ctypes.byref(d)) == 0
    # empty anchor set in view order: validated, nothing launched
    d = desc(Geo(), B=4, A=0)
    assert lib.msda_forward_workspace_size(ctypes.byref(d)) == 0
    assert lib.msda_forward_ws(FAKE, FAKE, FAKE, None, None, None, None, 0, ctypes.byref(d),
                               None) == _lib.MSDA_OK


def test_projection_validation(lib):
    d = _lib.MsdaProjDesc(1, 4, 3, 2, 0.1)
    expect(lib, lib.msda_project_keypoints(FAKE, FAKE, FAKE, FAKE, FAKE, None, ctypes.byref(d),
                                           None), INV, "NULL")
    bad = _lib.MsdaProjDesc(1, 4, 0, 2, 0.1)
    expect(lib, lib.msda_project_keypoints(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ctypes.byref(bad),
                                           None), INV, "positive")
    nan = _lib.MsdaProjDesc(1, 4, 3, 2, float("nan"))
    expect(lib, lib.msda_project_keypoints(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ctypes.byref(nan),
                                           None), INV, "NaN")
    big = _lib.MsdaProjDesc(1 << 10, 1 << 12, 13, 64, 0.0)
    expect(lib, lib.msda_project_keypoints(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ctypes.byref(big),
                                           None), UNS, "2^31")
    empty = _lib.MsdaProjDesc(1, 0, 3, 2, 0.0)
    assert lib.msda_project_keypoints(None, None, None, None, None, None, ctypes.byref(empty),
                                      None) == _lib.MSDA_OK


def test_visible_form_validation(lib):
    d = desc(Geo(), B=2, A=4, C=32)
    need_f = lib.msda_forward_visible_workspace_size(ctypes.byref(d))
    need_b = lib.msda_backward_visible_workspace_size(ctypes.byref(d))
    # compaction + one partial row per (batch item, camera, anchor)
    assert need_f >= 2 * 2 * 4 * 32 * 4
    assert need_b > lib.msda_backward_workspace_size(ctypes.byref(d))
    fwdv = lambda vis, ws, n: lib.msda_forward_visible(FAKE, FAKE, FAKE, FAKE, FAKE, vis,
                                                       FAKE + 4096, ws, n, ctypes.byref(d), None)
    expect(lib, fwdv(None, FAKE + (1 << 20), need_f), INV, "NULL")
    expect(lib, fwdv(FAKE, None, 0), WS, "workspace")
    expect(lib, fwdv(FAKE, FAKE + (1 << 20), need_f - 1), WS)
    bwdv = lambda vis, ws, n: lib.msda_backward_visible(FAKE, FAKE, FAKE, FAKE, FAKE, vis, FAKE,
                                                        FAKE + 8192, FAKE, FAKE, ws, n,
                                                        ctypes.byref(d), None)
    expect(lib, bwdv(None, FAKE + (1 << 20), need_b), INV, "visible")
    expect(lib, bwdv(FAKE, FAKE + (1 << 20), need_b - 1), WS)
    # anchor order cannot serve the visible-view form; nor can atomic grad_feat
    da = desc(Geo(), B=2, A=4, C=32, tile=(0, 0, _lib.MSDA_ORDER_ANCHOR, 0))
    expect(lib, lib.msda_forward_visible(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
                                         1 << 30, ctypes.byref(da), None), UNS, "view order")
    dt = desc(Geo(), B=2, A=4, C=32, tile=(0, 0, 0, _lib.MSDA_SCATTER_ATOMIC))
    expect(lib, lib.msda_backward_visible(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
                                          FAKE, FAKE, 1 << 30, ctypes.byref(dt), None), UNS,
           "sorted")
    # no anchors: nothing to do
    d0 = desc(Geo(), B=2, A=0, C=32)
    assert lib.msda_forward_visible(FAKE, FAKE, FAKE, None, None, None, None, None, 0,
                                    ctypes.byref(d0), None) == _lib.MSDA_OK


def test_fused_form_validation(lib):
    d = desc(Geo(), B=2, A=4, C=32)
    assert (lib.msda_forward_fused_workspace_size(ctypes.byref(d)) ==
            lib.msda_forward_visible_workspace_size(ctypes.byref(d)))
    assert (lib.msda_backward_fused_workspace_size(ctypes.byref(d)) ==
            lib.msda_backward_visible_workspace_size(ctypes.byref(d)))
    ws, n = FAKE + (1 << 20), 1 << 30
    # the forward needs the scores
    expect(lib, lib.msda_forward_fused(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE + 4096, ws,
                                       n, ctypes.byref(d), None), INV, "NULL")
    # the backward's score gradient needs the forward's output
    bwdf = lambda score, out, gs: lib.msda_backward_fused(
        FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, score, out, FAKE, FAKE + 8192, FAKE, FAKE, gs, ws, n,
        ctypes.byref(d), None)
    expect(lib, bwdf(None, FAKE, FAKE), INV, "view_score")
    expect(lib, bwdf(FAKE, None, FAKE), INV, "out")


def test_weight_flag_validation(lib):
    # an unknown flag bit
    expect(lib, fwd(lib, desc(Geo(), flags=64)), INV, "flags")
    # logits need the workspace for their softmax statistics
    d = desc(Geo(ncam=4), A=4, C=32, flags=_lib.MSDA_WEIGHT_LOGITS)
    expect(lib, fwd(lib, d), WS, "msda_forward_ws")
    plain = desc(Geo(ncam=4), A=4, C=32)
    assert (lib.msda_forward_workspace_size(ctypes.byref(d)) >
            lib.msda_forward_workspace_size(ctypes.byref(plain)))
    # the backward works on FP32 weights written once: 4 * G per sample more
    nsamp = 1 * 4 * 3 * 4 * 2
    for flags in (_lib.MSDA_WEIGHT_LOGITS, _lib.MSDA_WEIGHTS_BF16):
        df = desc(Geo(ncam=4), A=4, C=32, flags=flags)
        assert (lib.msda_backward_workspace_size(ctypes.byref(df)) >=
                lib.msda_backward_workspace_size(ctypes.byref(plain)) + 4 * 4 * nsamp)
    # the visible-view forms keep the softmax statistics in their workspaces
    dv = desc(Geo(), B=2, A=4, C=32, flags=_lib.MSDA_WEIGHT_LOGITS)
    pv = desc(Geo(), B=2, A=4, C=32)
    assert (lib.msda_forward_visible_workspace_size(ctypes.byref(dv)) >
            lib.msda_forward_visible_workspace_size(ctypes.byref(pv)))
    assert (lib.msda_backward_fused_workspace_size(ctypes.byref(dv)) >
            lib.msda_backward_fused_workspace_size(ctypes.byref(pv)))


def test_sort_validation(lib):
    n, mk = 5000, 1000
    ws = lib.msda_sort_workspace_size(n, mk)
    assert ws >= 4 * n * 4
    expect(lib, lib.msda_sort_keys(FAKE, n, mk, FAKE, None, FAKE, ws, None), INV)
    expect(lib, lib.msda_sort_keys(None, n, mk, FAKE, FAKE, FAKE, ws, None), INV)
    expect(lib, lib.msda_sort_keys(FAKE, n, 0xFFFFFFFF, FAKE, FAKE, FAKE, ws, None), INV,
           "max_key")
    expect(lib, lib.msda_sort_keys(FAKE, n, mk, FAKE, FAKE, FAKE, ws - 1, None), WS)
    expect(lib, lib.msda_sort_keys(FAKE, n, mk, FAKE, FAKE, FAKE + 16, ws, None), WS, "aligned")
    big = (1 << 31) + 1
    expect(lib, lib.msda_sort_keys(FAKE, big, mk, FAKE, FAKE, FAKE,
                                   lib.msda_sort_workspace_size(big, mk), None), INV, "2^31")
    # n == 0 needs no keys or order, only seg
    assert lib.msda_sort_workspace_size(0, mk) >= 0
    expect(lib, lib.msda_sort_keys(None, 0, mk, None, None, FAKE, 256, None), INV)
