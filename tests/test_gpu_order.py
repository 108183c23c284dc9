"""View order (MSDA_ORDER_VIEW): the (batch item, camera) x anchor work cut
into one range per XCD. Checked against the FP64 oracle on ragged shapes
and edge cases (fewer views than XCDs, view counts not divisible by 8,
single anchors, empty rows), and against anchor order: the backward's
outputs are per sample or per pair, so both orders give identical bits;
the forward adds in a different (fixed) order and agrees to rounding."""
import numpy as np
import pytest
import torch

from helpers import (BF16_TOL, FWD_F32_MAXREL, FWD_F32_TOL, GRAD_F32_MAXREL, GRAD_F32_TOL,
                     assert_close, host, normwise, to_device)
from paper_2601_10819_amd import synth

pytestmark = pytest.mark.gpu

VIEW = {"order": "view"}
ANCHOR = {"order": "anchor"}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ops():
    from paper_2601_10819_amd import ops as o
    o._lib.load()
    return o


CASES = [
    # (B, cams, levels, C, G, A, P, tile extras)
    (2, 7, ((11, 13), (6, 7), (3, 3)), 64, 4, 37, 5, {"waves_per_anchor": 4}),   # 14 views
    (3, 5, ((9, 10), (5, 5)), 32, 4, 11, 3, {"waves_per_anchor": 1}),           # 15 views
    (1, 3, ((7, 9), (4, 5)), 256, 8, 20, 4, {"waves_per_anchor": 8}),           # 3 views < 8
    (1, 16, ((8, 12), (4, 6), (2, 3), (1, 2)), 128, 8, 1, 13, {}),             # one anchor
    (2, 4, ((5, 7),), 16, 2, 9, 2, {"waves_per_anchor": 2, "chans_per_lane": 2}),
    (1, 9, tuple((9 - i, 10 - i) for i in range(8)), 32, 4, 6, 2, {}),          # 8 levels
]


def case_problem(i, B, cams, levels, C, G, A, P):
    return synth.small(seed=100 + i, B=B, cams=cams, levels=levels, C=C, G=G, A=A, P=P)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_view_order_matches_oracle(ops, oracle_mod, i):
    B, cams, levels, C, G, A, P, extra = CASES[i]
    p = case_problem(i, B, cams, levels, C, G, A, P)
    print(f"case {i} {p.dims()} {extra}", flush=True)
    feat, layout, loc, w = to_device(p)
    go = synth.grad_out_like(p, seed=i)
    tile = dict(VIEW, **extra)
    out = ops.forward(feat, layout, loc, w, tile=tile)
    gf, gl, gw = ops.backward(feat, layout, loc, w, go.cuda(), tile=tile)
    torch.cuda.synchronize()
    ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                             p.weights)
    assert_close(host(out), ref, FWD_F32_TOL, FWD_F32_MAXREL, f"case {i} out")
    rgf, rgl, rgw = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index,
                                        p.sampling_loc, p.weights, go)
    assert_close(host(gf), rgf, GRAD_F32_TOL, GRAD_F32_MAXREL, f"case {i} grad_feat")
    assert_close(host(gl), rgl, GRAD_F32_TOL, GRAD_F32_MAXREL, f"case {i} grad_loc")
    assert_close(host(gw), rgw, GRAD_F32_TOL, GRAD_F32_MAXREL, f"case {i} grad_w")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
def test_orders_agree(ops, dtype):
    """Backward: identical bits in both orders (and with the atomic grad_feat
    form switched off, records are the same). Forward: equal to rounding."""
    p = synth.small(seed=7, B=2, cams=12, levels=((16, 24), (8, 12), (4, 6), (2, 3)), C=256,
                    G=8, A=60, P=13)
    feat, layout, loc, w = to_device(p, dtype)
    go = synth.grad_out_like(p, seed=3).cuda()
    res = {}
    for name, tile in (("anchor", ANCHOR), ("view", VIEW)):
        out = ops.forward(feat, layout, loc, w, tile=tile)
        grads = ops.backward(feat, layout, loc, w, go, tile=tile)
        res[name] = (out,) + tuple(grads)
    torch.cuda.synchronize()
    for k, what in ((1, "grad_feat"), (2, "grad_loc"), (3, "grad_w")):
        assert torch.equal(res["anchor"][k], res["view"][k]), what
    assert normwise(host(res["view"][0]), host(res["anchor"][0])) <= 1e-6


def test_view_order_is_default_and_reproducible(ops):
    """With 8 or more views the library picks view order for ops.forward
    (which passes a workspace); repeated calls give identical bits, and the
    plain msda_forward (no workspace) runs anchor order."""
    p = synth.small(seed=9, B=1, cams=10, levels=((12, 20), (6, 10)), C=64, G=4, A=50, P=6)
    feat, layout, loc, w = to_device(p)
    assert ops.forward_workspace_bytes(feat, layout, loc, w) == 8 * 1 * 50 * 64 * 4
    a = ops.forward(feat, layout, loc, w)
    b = ops.forward(feat, layout, loc, w)
    v = ops.forward(feat, layout, loc, w, tile=VIEW)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, v)


def test_view_order_empty_and_all_out_of_range(ops):
    p = synth.small(seed=11, B=2, cams=6, A=1)
    feat, layout, loc, w = to_device(p)
    out = ops.forward(feat, layout, loc[:, :0].contiguous(), w[:, :0].contiguous(), tile=VIEW)
    torch.cuda.synchronize()
    assert out.shape == (2, 0, p.channels)
    p = synth.small(seed=12, B=2, cams=6, A=7, P=3)
    p.sampling_loc[..., 1] = -0.7
    feat, layout, loc, w = to_device(p)
    out = ops.forward(feat, layout, loc, w, tile=VIEW)
    gf, gl, gw = ops.backward(feat, layout, loc, w, torch.ones(2, 7, p.channels, device="cuda"),
                              tile=VIEW)
    torch.cuda.synchronize()
    assert torch.all(out == 0) and torch.all(gf == 0) and torch.all(gl == 0)
    assert torch.all(gw == 0)


def test_view_order_bf16_full_size_cam64(ops, oracle_mod):
    """The 64-camera workload in view order (the library's choice there),
    BF16 storage: a seeded anchor subset against the oracle on the stored
    values, forward and grad_w / grad_loc."""
    from helpers import anchor_subset, oracle_backward_subset, oracle_forward_subset
    p = synth.cam64()
    feat, layout, loc, w = to_device(p, torch.bfloat16)
    go = synth.grad_out_like(p, seed=2)
    out = ops.forward(feat, layout, loc, w, tile=VIEW)
    _, gl, gw = ops.backward(feat, layout, loc, w, go.cuda(), need_feat=False, tile=VIEW)
    torch.cuda.synchronize()
    idx = anchor_subset(p, 24, seed=5)
    feat64 = p.feat.to(torch.bfloat16).double()
    ref = oracle_forward_subset(oracle_mod, feat64, p, idx)
    assert_close(host(out)[:, idx], ref, FWD_F32_TOL, FWD_F32_MAXREL, "cam64 view out")
    rgl, rgw = oracle_backward_subset(oracle_mod, feat64, p, idx, go)
    assert_close(host(gl)[:, idx], rgl, GRAD_F32_TOL, GRAD_F32_MAXREL, "cam64 view grad_loc")
    assert_close(host(gw)[:, idx], rgw, GRAD_F32_TOL, GRAD_F32_MAXREL, "cam64 view grad_w")


@pytest.mark.parametrize("B,N,A,waves", [(1, 64, 900, 1), (1, 64, 900, 4), (2, 16, 1800, 2),
                                         (1, 6, 900, 4), (3, 7, 5, 1), (2, 3, 1, 8),
                                         (1, 1, 3, 2), (2, 9, 37, 4)])
def test_view_order_counts_every_item_once(ops, B, N, A, waves):
    """The view-order partition of the (batch item, camera, anchor) items over
    the XCD slots, checked through the library: channel n of every pixel of
    camera n is 1 (all other channels 0), every weight is 1 and every
    location is a pixel centre of the single level, so out[b, a, n] counts
    the samples of item (b, a, n) that the forward summed -- exactly P for
    every camera, none dropped or repeated -- and the backward's per-sample
    grad_w is 1 exactly where the camera's channel lies in the group, its
    grad_loc the exact one-sided difference."""
    C, G, P, H, W = 64, 16, 3, 4, 8
    shapes, starts, R = synth.layout([[(H, W)]] * N)
    feat = torch.zeros(B, R, C)
    for n in range(N):
        feat[:, starts[n, 0]:starts[n, 0] + H * W, n] = 1.0
    gen = torch.Generator().manual_seed(B * 1000 + N * 10 + A)
    ix = torch.randint(0, W, (B, A, P, N), generator=gen)
    iy = torch.randint(0, H, (B, A, P, N), generator=gen)
    loc = torch.stack([(ix + 0.5) / W, (iy + 0.5) / H], dim=-1)
    w = torch.ones(B, A, P, N, 1, G)
    layout = ops.Layout(shapes, starts)
    tile = {"order": "view", "waves_per_anchor": waves}
    feat, loc, w = feat.cuda(), loc.cuda(), w.cuda()
    out = ops.forward(feat, layout, loc, w, tile=tile)
    go = torch.ones(B, A, C, device="cuda")
    _, gl, gw = ops.backward(feat, layout, loc, w, go, need_feat=False, tile=tile)
    torch.cuda.synchronize()
    want = torch.zeros(B, A, C)
    want[..., :N] = float(P)
    assert torch.equal(out.cpu(), want)
    want_w = torch.zeros(B, A, P, N, 1, G)
    for n in range(N):
        want_w[:, :, :, n, 0, n // (C // G)] = 1.0
    assert torch.equal(gw.cpu(), want_w)
    # d out / d x at a pixel centre is the right-hand difference of the
    # camera's constant channel: 0 inside, -W (-H) at the last column (row),
    # where the right (lower) neighbour is zero padding
    want_l = torch.stack([torch.where(ix == W - 1, -float(W), 0.0),
                          torch.where(iy == H - 1, -float(H), 0.0)], dim=-1)
    assert torch.equal(gl.cpu(), want_l)
