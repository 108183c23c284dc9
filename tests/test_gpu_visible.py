"""Keypoint projection and the visible-view form of MSDA on the GPU against
the FP64 oracle: projection (locations and visibility), forward and
backward over visible pairs on ragged shapes and random masks, the dense
operator's bits for the per-pair gradients and grad_feat when every pair is
visible, empty masks, and the 64-camera outside-in scene end to end."""
import numpy as np
import pytest
import torch

from helpers import (FWD_F32_MAXREL, FWD_F32_TOL, GRAD_F32_MAXREL, GRAD_F32_TOL, anchor_subset,
                     assert_close, host, normwise, to_device)
from paper_2601_10819_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ops():
    from paper_2601_10819_amd import ops as o
    o._lib.load()
    return o


@pytest.fixture(scope="module")
def proj():
    from oracle import projection
    return projection


def geometry_to_device(g):
    return (g.anchors.cuda(), g.keypoints.cuda(), g.projection.cuda(), g.image_hw.cuda())


@pytest.mark.parametrize("cams,anchors,B", [(16, 200, 1), (7, 33, 2), (64, 60, 1)])
def test_projection_matches_oracle(ops, proj, cams, anchors, B):
    g = synth.outside_in(seed=cams, B=B, cams=cams, anchors=anchors)
    print(f"case cams={cams} anchors={anchors} B={B}", flush=True)
    loc, vis = ops.project_keypoints(*geometry_to_device(g), g.dt)
    torch.cuda.synchronize()
    rloc, rvis = proj.project_keypoints(g.anchors, g.keypoints, g.dt, g.projection, g.image_hw)
    loc, vis = host(loc), host(vis).astype(bool)
    behind = rloc[..., 0] == proj.BEHIND
    assert np.array_equal(loc[..., 0] == proj.BEHIND, behind)
    # normalised locations: FP32 world coordinates (metres) and matrices
    # give ~1e-6 relative; 2e-5 of the image is ~0.01 px. Points near a
    # camera's focal plane are ill-conditioned (tiny depth) and land far
    # outside the image: there, both sides must agree that the point is
    # beyond every level (outside [-0.05, 1.05]), which is all MSDA uses.
    near = ~behind & (np.abs(rloc - 0.5) <= 0.6).all(-1)
    np.testing.assert_allclose(loc[near], rloc[near], atol=2e-5, rtol=0)
    far = (~behind)[..., None] & (np.abs(rloc - 0.5) > 0.56)
    assert np.all(np.abs(loc[far] - 0.5) > 0.55)
    # visibility is decided by comparisons: compare where no keypoint of the
    # pair lies within 0.05 px of an image edge (where FP32 and FP64 may
    # decide differently)
    pts = proj.keypoints_world(g.anchors, g.keypoints, g.dt)
    pix, depth = proj.project_points(pts, g.projection, g.image_hw)
    hw = g.image_hw.numpy().astype(np.float64)
    H, W = hw[:, 0][None, None, None], hw[:, 1][None, None, None]
    edge = (np.minimum.reduce([np.abs(pix[..., 0]), np.abs(pix[..., 0] - W),
                               np.abs(pix[..., 1]), np.abs(pix[..., 1] - H)]) < 0.05) & \
        (depth > proj.DEPTH_EPS)
    ambiguous = edge.any(axis=2)
    assert np.array_equal(vis[~ambiguous], rvis[~ambiguous])
    assert 0.05 < rvis.mean() < 0.95


CASES = [
    # (seed, B, cams, levels, C, G, A, P, density)
    (0, 2, 7, ((11, 13), (6, 7), (3, 3)), 64, 4, 37, 5, 0.3),
    (1, 1, 12, ((9, 10), (5, 5)), 32, 4, 25, 3, 0.1),
    (2, 1, 3, ((7, 9), (4, 5)), 256, 8, 20, 4, 0.7),
    (3, 3, 5, ((8, 12), (4, 6), (2, 3), (1, 2)), 128, 8, 9, 13, 0.5),
]


def case_problem(c):
    seed, B, cams, levels, C, G, A, P, dens = c
    p = synth.small(seed=200 + seed, B=B, cams=cams, levels=levels, C=C, G=G, A=A, P=P)
    rng = np.random.default_rng(seed)
    vis = rng.random((B, A, cams)) < dens
    return p, vis


@pytest.mark.parametrize("i", range(len(CASES)))
def test_visible_forward_backward_match_oracle(ops, proj, i):
    p, vis = case_problem(CASES[i])
    print(f"case {i} {p.dims()} density {vis.mean():.2f}", flush=True)
    feat, layout, loc, w = to_device(p)
    v = torch.from_numpy(vis.astype(np.uint8)).cuda()
    go = synth.grad_out_like(p, seed=i)
    out = ops.forward_visible(feat, layout, loc, w, v)
    gf, gl, gw = ops.backward_visible(feat, layout, loc, w, v, go.cuda())
    torch.cuda.synchronize()
    ref = proj.forward_visible(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights, vis)
    assert_close(host(out), ref, FWD_F32_TOL, FWD_F32_MAXREL, f"case {i} out")
    rgf, rgl, rgw = proj.backward_visible(p.feat, p.spatial_shapes, p.level_start_index,
                                          p.sampling_loc, p.weights, vis, go.numpy())
    assert_close(host(gf), rgf, GRAD_F32_TOL, GRAD_F32_MAXREL, f"case {i} grad_feat")
    assert_close(host(gl), rgl, GRAD_F32_TOL, GRAD_F32_MAXREL, f"case {i} grad_loc")
    assert_close(host(gw), rgw, GRAD_F32_TOL, GRAD_F32_MAXREL, f"case {i} grad_w")
    # invisible pairs: exactly zero
    inv = ~vis
    assert np.all(host(gw)[np.broadcast_to(inv[:, :, None, :, None, None], rgw.shape)] == 0)
    assert np.all(host(gl)[np.broadcast_to(inv[:, :, None, :, None], rgl.shape)] == 0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float16],
                         ids=["f32", "bf16", "f16"])
def test_all_visible_equals_dense(ops, dtype):
    """Every pair visible: grad_w, grad_loc and grad_feat are the dense
    operator's bits (same per-pair arithmetic, same record order within each
    cell); the forward agrees to rounding (it adds cameras in another order)."""
    p = synth.small(seed=31, B=2, cams=9, levels=((16, 24), (8, 12), (4, 6), (2, 3)), C=256, G=8,
                    A=40, P=13)
    feat, layout, loc, w = to_device(p, dtype)
    v = torch.ones(2, 40, 9, dtype=torch.uint8, device="cuda")
    go = synth.grad_out_like(p, seed=5).cuda()
    out_v = ops.forward_visible(feat, layout, loc, w, v)
    g_v = ops.backward_visible(feat, layout, loc, w, v, go)
    out_d = ops.forward(feat, layout, loc, w, tile={"order": "view"})
    g_d = ops.backward(feat, layout, loc, w, go, tile={"order": "view"})
    torch.cuda.synchronize()
    for a, b, what in zip(g_v, g_d, ("grad_feat", "grad_loc", "grad_w")):
        assert torch.equal(a, b), what
    assert normwise(host(out_v), host(out_d)) <= 1e-6


@pytest.mark.parametrize("which", ["cam64", "train16"])
def test_bucket_sort_equals_global_sort(ops, which):
    """The backward sorts its records per (batch item, region) bucket in LDS;
    MSDA_SCATTER_SORTED_GLOBAL sorts the same records with the global radix
    sort instead. Every cell must list the same records in the same order,
    so grad_feat is bitwise the same -- dense, and in the visible-view form
    with every pair visible (which equals the dense form) -- at the
    64-camera scene's bucket size (11,700 records) and the 16-camera training
    workload (2 batch items, 23,400 per bucket, a quarter of them outside
    every level), BF16."""
    p = synth.cam64(seed=2, anchors=900, cams=16) if which == "cam64" else synth.train16(seed=2)
    print(f"bucket vs global sort: {p.name} {p.dims()}", flush=True)
    feat, layout, loc, w = to_device(p, torch.bfloat16)
    v = torch.ones(p.batch, p.num_anchors, p.num_cams, dtype=torch.uint8, device="cuda")
    go = synth.grad_out_like(p, seed=5).cuda()
    glob = {"scatter": _lib.MSDA_SCATTER_SORTED_GLOBAL}
    gf_v, _, _ = ops.backward_visible(feat, layout, loc, w, v, go)
    gf_vg, _, _ = ops.backward_visible(feat, layout, loc, w, v, go, tile=glob)
    gf_d, _, _ = ops.backward(feat, layout, loc, w, go, need_loc=False, need_w=False,
                              tile={"order": "view"})
    gf_dg, _, _ = ops.backward(feat, layout, loc, w, go, need_loc=False, need_w=False,
                               tile=dict(glob, order="view"))
    torch.cuda.synchronize()
    assert torch.equal(gf_d, gf_dg), "dense: bucket vs global"
    assert torch.equal(gf_v, gf_vg), "visible: bucket vs global"
    assert torch.equal(gf_v, gf_d), "visible (all) vs dense"


@pytest.mark.parametrize("fused", [False, True], ids=["visible", "fused"])
def test_visible_buckets_equal_global_sort(ops, fused):
    """Visible-view records bucketed per (batch item, camera, level) from the
    visible-item scan: regions receive uneven record counts (a camera sees
    none, one sees every anchor, the rest about a quarter), and the bucketed
    sort must give every output bitwise equal to the global radix sort's --
    for the visible-view and the fused form, B = 2, BF16."""
    p = synth.small(seed=81, B=2, cams=12, levels=((24, 40), (12, 20), (6, 10), (3, 5)),
                    C=256, G=8, A=300, P=13)
    print(f"visible buckets: {p.dims()} fused={fused}", flush=True)
    feat, layout, loc, w = to_device(p, torch.bfloat16)
    gen = torch.Generator().manual_seed(82)
    v = (torch.rand(p.batch, p.num_anchors, p.num_cams, generator=gen) < 0.25).to(torch.uint8)
    v[:, :, 3] = 0
    v[:, :, 7] = 1
    v = v.cuda()
    go = synth.grad_out_like(p, seed=83).cuda()
    glob = {"scatter": _lib.MSDA_SCATTER_SORTED_GLOBAL}
    if fused:
        score = torch.rand(p.batch, p.num_anchors, p.num_cams, generator=gen).cuda()
        out = ops.forward_fused(feat, layout, loc, w, v, score)
        g_b = ops.backward_fused(feat, layout, loc, w, v, score, out, go)
        g_g = ops.backward_fused(feat, layout, loc, w, v, score, out, go, tile=glob)
    else:
        g_b = ops.backward_visible(feat, layout, loc, w, v, go)
        g_g = ops.backward_visible(feat, layout, loc, w, v, go, tile=glob)
    torch.cuda.synchronize()
    assert len(g_b) == len(g_g)
    for i, (a, b) in enumerate(zip(g_b, g_g)):
        assert torch.equal(a, b), f"output {i}"


def test_nothing_visible(ops):
    p = synth.small(seed=33, B=1, cams=4, A=6, P=3)
    feat, layout, loc, w = to_device(p)
    v = torch.zeros(1, 6, 4, dtype=torch.uint8, device="cuda")
    out = ops.forward_visible(feat, layout, loc, w, v)
    gf, gl, gw = ops.backward_visible(feat, layout, loc, w, v,
                                      torch.ones(1, 6, p.channels, device="cuda"))
    torch.cuda.synchronize()
    assert torch.all(out == 0) and torch.all(gf == 0) and torch.all(gl == 0)
    assert torch.all(gw == 0)


def test_outside_in_64cam_end_to_end(ops, proj, oracle_mod):
    """Projection on the GPU feeding the visible-view forward and backward
    (BF16 features) on the 64-camera scene: seeded anchor subsets against the
    oracle on the projected locations, and the Euler identities."""
    g = synth.outside_in(seed=0, cams=64, anchors=900)
    p = synth.cam64()
    loc, vis = ops.project_keypoints(*geometry_to_device(g), g.dt)
    feat = p.feat.to(torch.bfloat16).cuda()
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    w = p.weights.cuda()
    go = synth.grad_out_like(p, seed=9).cuda()
    out = ops.forward_visible(feat, layout, loc, w, vis)
    gf, gl, gw = ops.backward_visible(feat, layout, loc, w, vis, go)
    torch.cuda.synchronize()
    vis_h = host(vis).astype(bool)
    print(f"visible pairs {vis_h.mean():.3f}", flush=True)
    idx = anchor_subset(p, 16, seed=3)
    loc_h = torch.from_numpy(host(loc))
    feat64 = p.feat.to(torch.bfloat16).double()
    ref = proj.forward_visible(feat64, p.spatial_shapes, p.level_start_index,
                               loc_h[:, idx].contiguous(), p.weights[:, idx].contiguous(),
                               vis_h[:, idx])
    assert_close(host(out)[:, idx], ref, FWD_F32_TOL, FWD_F32_MAXREL, "64cam visible out")
    e_out = float((out.double() * go.double()).sum())
    pw = float((gw.double() * w.double()).sum())
    assert abs(pw - e_out) <= 1e-5 * float((gw.double() * w.double()).abs().sum())
    pf = gf.double() * feat.double()
    assert abs(float(pf.sum()) - e_out) <= 2.0 ** -9 * float(pf.abs().sum())
