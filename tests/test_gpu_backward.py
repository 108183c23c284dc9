"""Backward parity of the HIP kernels: FP32 gradients against the FP64
oracle's analytic gradient and against central finite differences; Euler
identities at full size; the autograd wrapper."""
import numpy as np
import pytest
import torch

from helpers import (BF16_TOL, GRAD_F32_MAXREL, GRAD_F32_TOL, anchor_subset, assert_close,
                     host, normwise, oracle_backward_subset, to_device)
from paper_2601_10819_amd import synth

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


def run_bwd(ops, p, go, dtype=torch.float32, tile=None, **kw):
    feat, layout, loc, w = to_device(p, dtype)
    gf, gl, gw = ops.backward(feat, layout, loc, w, go.cuda(), tile=tile, **kw)
    torch.cuda.synchronize()
    return tuple(None if t is None else host(t) for t in (gf, gl, gw))


def check_all(got, ref, what):
    for name, g, r in zip(("grad_feat", "grad_loc", "grad_w"), got, ref):
        assert_close(g, r, GRAD_F32_TOL, GRAD_F32_MAXREL, f"{what} {name}")


@pytest.mark.parametrize("maker", [synth.tiny, lambda: synth.sparse4d(seed=0)],
                         ids=["tiny_2cam_c64", "sparse4d_6cam"])
def test_backward_matches_oracle(ops, oracle_mod, maker):
    p = maker()
    print(f"case {p.name} {p.dims()}", flush=True)
    go = synth.grad_out_like(p, seed=1)
    got = run_bwd(ops, p, go)
    ref = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, go)
    check_all(got, ref, p.name)


@pytest.mark.parametrize("C,G,cpl,waves", [
    (256, 8, 4, 1), (256, 8, 4, 4), (128, 8, 2, 2), (64, 8, 1, 8), (64, 4, 4, 2),
    (32, 4, 2, 1), (16, 2, 4, 4), (4, 1, 4, 1),
])
def test_backward_lane_layouts(ops, oracle_mod, C, G, cpl, waves):
    p = synth.small(seed=100 + C + waves, B=2, cams=5, levels=((11, 13), (6, 7), (3, 3)), C=C,
                    G=G, A=23, P=5)
    print(f"case C={C} G={G} cpl={cpl} waves={waves}", flush=True)
    go = synth.grad_out_like(p, seed=2)
    got = run_bwd(ops, p, go, tile={"chans_per_lane": cpl, "waves_per_anchor": waves})
    ref = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, go)
    check_all(got, ref, f"C={C} cpl={cpl} waves={waves}")


def test_backward_partial_requests_and_out_of_range(ops, oracle_mod):
    p = synth.small(seed=7, A=11, P=4, loc_mode="out_of_view")
    go = synth.grad_out_like(p, seed=3)
    ref = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, go)
    for need in [(True, False, False), (False, True, False), (False, False, True)]:
        got = run_bwd(ops, p, go, need_feat=need[0], need_loc=need[1], need_w=need[2])
        for want, g, r in zip(need, got, ref):
            if want:
                assert_close(g, r, GRAD_F32_TOL, GRAD_F32_MAXREL, "partial")
            else:
                assert g is None
    # all samples outside: every gradient is exactly zero
    p.sampling_loc[..., 1] = -0.75
    gf, gl, gw = run_bwd(ops, p, go)
    assert np.all(gf == 0) and np.all(gl == 0) and np.all(gw == 0)


def test_grad_loc_matches_finite_differences(ops, oracle_mod):
    """GPU grad_sampling_loc against central differences of the FP64 oracle
    forward (h = 1e-7; locations >= 1e-3 px from grid lines)."""
    p = synth.sparse4d(seed=0)
    go = synth.grad_out_like(p, seed=4)
    _, gl, _ = run_bwd(ops, p, go, need_feat=False, need_w=False)
    rng = np.random.default_rng(5)
    feat = p.feat.double().numpy()
    loc = p.sampling_loc.double().numpy()
    w = p.weights.double().numpy()
    gon = go.double().numpy()
    fd, an = [], []
    for _ in range(40):
        a, pp, n, k = (int(rng.integers(0, s)) for s in (p.num_anchors, p.num_points,
                                                          p.num_cams, 2))
        lp = loc[:, a:a + 1].copy()
        lm = lp.copy()
        lp[0, 0, pp, n, k] += 1e-7
        lm[0, 0, pp, n, k] -= 1e-7
        op = oracle_mod.forward(feat, p.spatial_shapes, p.level_start_index, lp, w[:, a:a + 1])
        om = oracle_mod.forward(feat, p.spatial_shapes, p.level_start_index, lm, w[:, a:a + 1])
        fd.append(float(((op - om)[0, 0] * gon[0, a]).sum()) / 2e-7)
        an.append(gl[0, a, pp, n, k])
    assert_close(np.array(an), np.array(fd), GRAD_F32_TOL, None, "grad_loc vs FD")


@pytest.mark.parametrize("which", ["train16", "cam64"])
def test_backward_full_size(ops, oracle_mod, which):
    """Full-size workloads (default launch shape, FP32 storage): grad_loc and
    grad_w on a seeded anchor subset vs the oracle; grad_feat via the Euler
    identities <grad_feat, feat> = <grad_out, out> = <grad_w, w>."""
    p = synth.train16() if which == "train16" else synth.cam64()
    print(f"case {p.name} {p.dims()}", flush=True)
    go = synth.grad_out_like(p, seed=5)
    feat, layout, loc, w = to_device(p)
    out = ops.forward(feat, layout, loc, w)
    gf, gl, gw = ops.backward(feat, layout, loc, w, go.cuda())
    torch.cuda.synchronize()
    idx = anchor_subset(p, 32, seed=2)
    rgl, rgw = oracle_backward_subset(oracle_mod, p.feat, p, idx, go)
    assert_close(host(gl)[:, idx], rgl, GRAD_F32_TOL, GRAD_F32_MAXREL, "grad_loc")
    assert_close(host(gw)[:, idx], rgw, GRAD_F32_TOL, GRAD_F32_MAXREL, "grad_w")
    e_out = float((out.double() * go.cuda().double()).sum())
    e_feat = float((gf.double() * feat.double()).sum())
    e_w = float((gw.double() * w.double()).sum())
    assert abs(e_feat - e_out) <= 1e-5 * abs(e_out), (e_feat, e_out)
    assert abs(e_w - e_out) <= 1e-5 * abs(e_out), (e_w, e_out)


def test_grad_feat_full_size_cam64(ops, oracle_mod):
    """grad_feat at the 64-camera workload against the full oracle backward."""
    p = synth.cam64()
    go = synth.grad_out_like(p, seed=6)
    gf, _, _ = run_bwd(ops, p, go, need_loc=False, need_w=False)
    rgf, _, _ = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index,
                                    p.sampling_loc, p.weights, go, need_loc=False, need_w=False)
    assert_close(gf, rgf, GRAD_F32_TOL, GRAD_F32_MAXREL, "grad_feat cam64")


def test_autograd_function(ops, oracle_mod):
    p = synth.small(seed=9, B=2, cams=3, C=64, G=4, A=13, P=4)
    feat, layout, loc, w = to_device(p)
    feat.requires_grad_(True)
    loc.requires_grad_(True)
    w.requires_grad_(True)
    out = ops.msda(feat, layout, loc, w)
    go = synth.grad_out_like(p, seed=10).cuda()
    (out * go).sum().backward()
    torch.cuda.synchronize()
    ref = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, go.cpu())
    check_all((host(feat.grad), host(loc.grad), host(w.grad)), ref, "autograd")
    # a leaf that does not require grad receives none
    loc2 = loc.detach()
    feat2 = feat.detach().requires_grad_(True)
    ops.msda(feat2, layout, loc2, w.detach()).sum().backward()
    assert feat2.grad is not None and loc2.grad is None


def test_autograd_training_step_train16_bf16(ops, oracle_mod):
    """The outside-in training step (B = 2, 16 cameras, BF16 features, FP32
    locations and weights, 25% of keypoints outside each camera's view)
    through the autograd Function with loss = <grad_out, out>: the forward on
    an anchor subset, feat.grad in full, loc.grad and w.grad on an anchor
    subset, each against the oracle on the stored (widened) features, plus
    the Euler identities of the whole step."""
    p = synth.train16()
    print(f"case {p.name} {p.dims()} bf16 autograd", flush=True)
    go = synth.grad_out_like(p, seed=11)
    feat, layout, loc, w = to_device(p, torch.bfloat16)
    feat.requires_grad_(True)
    loc.requires_grad_(True)
    w.requires_grad_(True)
    out = ops.msda(feat, layout, loc, w)
    loss = (out * go.cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert feat.grad.dtype == torch.bfloat16
    assert loc.grad.dtype == torch.float32 and w.grad.dtype == torch.float32
    feat64 = p.feat.to(torch.bfloat16).double()
    idx = anchor_subset(p, 48, seed=12)
    ref_out = oracle_mod.forward(feat64, p.spatial_shapes, p.level_start_index,
                                 p.sampling_loc[:, idx].contiguous(),
                                 p.weights[:, idx].contiguous())
    assert_close(host(out)[:, idx], ref_out, 1e-5, 2e-4, "train16 bf16 out")
    rgl, rgw = oracle_backward_subset(oracle_mod, feat64, p, idx, go)
    assert_close(host(loc.grad)[:, idx], rgl, GRAD_F32_TOL, GRAD_F32_MAXREL, "train16 loc.grad")
    assert_close(host(w.grad)[:, idx], rgw, GRAD_F32_TOL, GRAD_F32_MAXREL, "train16 w.grad")
    # the out-of-view samples (a quarter of the keypoint-camera pairs) give
    # exact zeros in loc.grad
    u = p.sampling_loc[..., 0]
    v = p.sampling_loc[..., 1]
    outside = ((u < -0.4) | (u > 1.4) | (v < -0.4) | (v > 1.4)).cuda()
    assert 0.2 < float(outside.double().mean()) < 0.3
    assert torch.all(loc.grad[outside] == 0)
    rgf, _, _ = oracle_mod.backward(feat64, p.spatial_shapes, p.level_start_index,
                                    p.sampling_loc, p.weights, go, need_loc=False, need_w=False)
    gf = host(feat.grad)
    assert normwise(gf, rgf) <= BF16_TOL
    rounded = torch.from_numpy(rgf).float().to(torch.bfloat16).double().numpy()
    assert normwise(gf, rounded) <= 5e-3
    assert np.mean(gf == rounded) >= 0.99
    e_out = float(loss.double())
    pf = feat.grad.double() * feat.detach().double()
    pw = w.grad.double() * w.detach().double()
    assert abs(float(pf.sum()) - e_out) <= 2.0 ** -9 * float(pf.abs().sum()), e_out
    assert abs(float(pw.sum()) - e_out) <= 1e-5 * float(pw.abs().sum()), e_out


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float16],
                         ids=["f32", "bf16", "f16"])
def test_sorted_grad_feat_is_bitwise_reproducible(ops, oracle_mod, dtype):
    """The default (sorted) grad_feat sums each row in sample order: repeated
    calls and different launch shapes give identical bits, and both it and
    the float-atomic form match the oracle."""
    p = synth.sparse4d(seed=3, anchors=300)
    go = synth.grad_out_like(p, seed=8).cuda()
    feat, layout, loc, w = to_device(p, dtype)
    runs = []
    for tile in [None, {"waves_per_anchor": 1}, {"waves_per_anchor": 8},
                 {"waves_per_anchor": 2, "chans_per_lane": 4}, {"order": "view"},
                 {"order": "view", "waves_per_anchor": 8}, None]:
        gf, _, _ = ops.backward(feat, layout, loc, w, go, need_loc=False, need_w=False,
                                tile=tile, deterministic=True)
        runs.append(gf)
    torch.cuda.synchronize()
    for r in runs[1:]:
        assert torch.equal(r, runs[0])
    ref_feat = p.feat.to(dtype).double()
    rgf, _, _ = oracle_mod.backward(ref_feat, p.spatial_shapes, p.level_start_index,
                                    p.sampling_loc, p.weights, go.cpu(), need_loc=False,
                                    need_w=False)
    tol = GRAD_F32_TOL if dtype == torch.float32 else BF16_TOL
    assert_close(host(runs[0]), rgf, tol, None, "sorted grad_feat")
    ga, _, _ = ops.backward(feat, layout, loc, w, go, need_loc=False, need_w=False,
                            tile={"scatter": 2})
    torch.cuda.synchronize()
    assert_close(host(ga), rgf, tol, None, "atomic grad_feat")


def test_sorted_grad_feat_hot_pixels(ops, oracle_mod):
    """Every sample of every anchor on the same few pixels: segments of
    thousands of records per row."""
    p = synth.small(seed=12, cams=2, levels=((6, 8), (3, 4)), C=64, G=4, A=150, P=13)
    gen = torch.Generator().manual_seed(4)
    # 3 distinct points shared by all anchors and keypoints
    pts = torch.tensor([[0.31, 0.42], [0.55, 0.61], [0.8, 0.2]])
    choice = torch.randint(0, 3, p.sampling_loc.shape[:-1], generator=gen)
    p.sampling_loc.copy_(pts[choice])
    go = synth.grad_out_like(p, seed=9)
    gf, gl, gw = run_bwd(ops, p, go)
    ref = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, go)
    check_all((gf, gl, gw), ref, "hot pixels")
