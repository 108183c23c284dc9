"""Forward parity of the HIP kernels against the FP64 oracle (FP32 storage),
over every lane layout and wave split, ragged shapes and edge cases."""
import numpy as np
import pytest
import torch

from helpers import (FWD_F32_MAXREL, FWD_F32_TOL, GRAD_F32_MAXREL, GRAD_F32_TOL, anchor_subset,
                     assert_close, host, oracle_forward_subset, to_device)
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


def run_fwd(ops, p, dtype=torch.float32, tile=None):
    feat, layout, loc, w = to_device(p, dtype)
    out = ops.forward(feat, layout, loc, w, tile=tile)
    torch.cuda.synchronize()
    return host(out)


@pytest.mark.parametrize("maker", [synth.tiny, lambda: synth.sparse4d(seed=0)],
                         ids=["tiny_2cam_c64", "sparse4d_6cam"])
def test_forward_matches_oracle(ops, oracle_mod, maker):
    p = maker()
    print(f"case {p.name} {p.dims()}", flush=True)
    got = run_fwd(ops, p)
    ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                             p.weights)
    assert_close(got, ref, FWD_F32_TOL, FWD_F32_MAXREL, p.name)


LAYOUTS = [
    # (C, G, chans_per_lane, waves_per_anchor)
    (256, 8, 4, 1), (256, 8, 4, 2), (256, 8, 4, 8), (128, 8, 2, 4), (64, 8, 1, 2),
    (64, 4, 4, 1), (64, 4, 2, 2), (32, 4, 4, 4), (16, 2, 4, 1), (8, 1, 1, 8), (4, 1, 4, 2),
]


@pytest.mark.parametrize("C,G,cpl,waves", LAYOUTS)
def test_forward_lane_layouts(ops, oracle_mod, C, G, cpl, waves):
    """Ragged shapes (odd H/W, 3 levels, 5 keypoints, 7 cameras) under every
    channels-per-lane / waves split the F32 kernel is built for."""
    p = synth.small(seed=C + waves, B=2, cams=7, levels=((11, 13), (6, 7), (3, 3)), C=C, G=G,
                    A=37, P=5)
    print(f"case C={C} G={G} cpl={cpl} waves={waves}", flush=True)
    got = run_fwd(ops, p, tile={"chans_per_lane": cpl, "waves_per_anchor": waves})
    ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                             p.weights)
    assert_close(got, ref, FWD_F32_TOL, FWD_F32_MAXREL, f"C={C} cpl={cpl} waves={waves}")


def test_forward_edge_cases(ops, oracle_mod):
    # every sample out of range -> exact zeros
    p = synth.small(seed=3, A=9, P=4)
    p.sampling_loc[..., 0] = 1.5
    assert np.all(run_fwd(ops, p) == 0.0)
    # one level, one camera, one keypoint, one channel group
    p = synth.small(seed=4, cams=1, levels=((5, 3),), C=8, G=1, A=3, P=1)
    ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc, p.weights)
    assert_close(run_fwd(ops, p), ref, FWD_F32_TOL, FWD_F32_MAXREL, "single")
    # 1x1 levels (every in-range sample touches the only pixel)
    p = synth.small(seed=5, cams=2, levels=((1, 1), (1, 2)), C=16, G=2, A=5, P=3)
    ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc, p.weights)
    assert_close(run_fwd(ops, p), ref, FWD_F32_TOL, FWD_F32_MAXREL, "1x1")
    # 8 levels (two blocks of four in the kernel)
    p = synth.small(seed=6, cams=2, levels=tuple((9 - i, 10 - i) for i in range(8)), C=32, G=4,
                    A=6, P=2)
    ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc, p.weights)
    assert_close(run_fwd(ops, p), ref, FWD_F32_TOL, FWD_F32_MAXREL, "8 levels")


def test_forward_empty_anchor_set(ops):
    p = synth.small(seed=1, A=1)
    feat, layout, loc, w = to_device(p)
    out = ops.forward(feat, layout, loc[:, :0].contiguous(), w[:, :0].contiguous())
    torch.cuda.synchronize()
    assert out.shape == (1, 0, p.channels)
    # the backward of an empty anchor set still writes grad_feat (all zero)
    gf, gl, gw = ops.backward(feat, layout, loc[:, :0].contiguous(), w[:, :0].contiguous(),
                              torch.zeros(1, 0, p.channels, device="cuda"))
    torch.cuda.synchronize()
    assert torch.all(gf == 0) and gl.numel() == 0 and gw.numel() == 0


def test_forward_pixel_centres_exact(ops):
    """u = (i + 0.5) / W with power-of-two W hits pixel i exactly: the output
    equals weight * feature bit for bit (one nonzero weight per anchor)."""
    gen = torch.Generator().manual_seed(11)
    levels = [(16, 32), (8, 16)]
    shapes, starts, R = synth.layout([levels] * 3)
    B, A, P, N, L, G, C = 1, 40, 1, 3, 2, 4, 64
    feat = torch.randn(B, R, C, generator=gen)
    ix = torch.randint(0, 32, (B, A, P, N), generator=gen)
    iy = torch.randint(0, 16, (B, A, P, N), generator=gen)
    loc = torch.stack([(ix + 0.5) / 32, (iy + 0.5) / 16], dim=-1).float().contiguous()
    w = torch.zeros(B, A, P, N, L, G)
    w[:, :, 0, 1, 0, :] = 1.0
    p = synth.Problem("centres", feat, shapes, starts, loc, w)
    got = run_fwd(ops, p)
    rows = starts[1, 0].item() + iy[0, :, 0, 1] * 32 + ix[0, :, 0, 1]
    assert np.array_equal(got[0], feat[0, rows].double().numpy())


def _affine_feat(shapes, starts, R, C, gen, centre=30):
    """FP32 features on the GPU, affine in each level's pixel coordinates:
    F[start + y*W + x, c] = alpha_c + beta_c * (x - xc) + gamma_c * (y - yc)
    with (xc, yc) = (W, H) - centre (small integers, exact in FP32), so every
    interior bilinear sample is exact. Centred on the sampled corner of the
    level, the values stay about 100 there, like a feature map's (the FP32
    difference of neighbouring corners that grad_sampling_loc takes would
    otherwise cancel digits)."""
    alpha = torch.randint(-50, 50, (C,), generator=gen).float()
    beta = torch.randint(-3, 4, (C,), generator=gen).float()
    gamma = torch.randint(-3, 4, (C,), generator=gen).float()
    feat = torch.zeros(1, R, C, device="cuda")
    a, b, g = alpha.cuda(), beta.cuda(), gamma.cuda()
    for n in range(shapes.shape[0]):
        H, W = int(shapes[n, 0, 0]), int(shapes[n, 0, 1])
        s0 = int(starts[n, 0])
        ys = torch.arange(H, device="cuda", dtype=torch.float32) - (H - centre)
        xs = torch.arange(W, device="cuda", dtype=torch.float32) - (W - centre)
        for y0 in range(0, H, 256):                      # a band of rows at a time
            yb = ys[y0:y0 + 256]
            blk = a + b * xs[None, :, None] + g * yb[:, None, None]
            feat[0, s0 + y0 * W:s0 + (y0 + len(yb)) * W] = blk.reshape(-1, C)
    return feat, alpha.double(), beta.double(), gamma.double()


def _interior_locs(shapes, A, P, gen, margin=60):
    """(u, v) whose four corners lie inside the level, in its last `margin`
    rows and columns (the highest offsets of each camera)."""
    N = shapes.shape[0]
    loc = torch.empty(1, A, P, N, 2)
    for n in range(N):
        H, W = int(shapes[n, 0, 0]), int(shapes[n, 0, 1])
        x = W - margin + torch.rand(A, P, generator=gen) * (margin - 2)
        y = H - margin + torch.rand(A, P, generator=gen) * (margin - 2)
        loc[0, :, :, n, 0] = (x + 0.5) / W
        loc[0, :, :, n, 1] = (y + 0.5) / H
    return loc


def test_forward_backward_beyond_2gib(ops):
    """One batch item of 4.19 GB of FP32 features (2 cameras x one 1024 x 2000
    level, C = 256), beyond 2^31 bytes and close to the 4 GiB limit, with
    samples in each camera's last rows: the output, grad_weights and
    grad_sampling_loc against closed forms (affine features are interpolated
    exactly; d/dx of the sample is beta, d/dy gamma), and grad_feat by the
    identity <grad_feat, feat> = <grad_out, out>."""
    C, G, A, P = 256, 8, 24, 4
    shapes, starts, R = synth.layout([[(1024, 2000)]] * 2)
    assert 2 ** 31 < R * C * 4 <= 2 ** 32 - 8192
    gen = torch.Generator().manual_seed(7)
    feat, alpha, beta, gamma = _affine_feat(shapes, starts, R, C, gen)
    loc = _interior_locs(shapes, A, P, gen)
    w = torch.rand(1, A, P, 2, 1, G, generator=gen)
    go = torch.randn(1, A, C, generator=gen)
    layout = ops.Layout(shapes, starts)
    print(f"beyond 2 GiB: R={R} bytes={R * C * 4}", flush=True)
    out = ops.forward(feat, layout, loc.cuda(), w.cuda())
    gf, gl, gw = ops.backward(feat, layout, loc.cuda(), w.cuda(), go.cuda())
    torch.cuda.synchronize()
    # closed forms in FP64
    Wd = shapes[:, 0, 1].double()[None, None, :]
    Hd = shapes[:, 0, 0].double()[None, None, :]
    x = loc[0, ..., 0].double() * Wd - 0.5                   # [A, P, N]
    y = loc[0, ..., 1].double() * Hd - 0.5
    xc, yc = Wd - 30, Hd - 30                                 # the map's centre
    val = alpha + beta * (x - xc)[..., None] + gamma * (y - yc)[..., None]   # [A, P, N, C]
    wc = w[0, :, :, :, 0].double().repeat_interleave(C // G, dim=-1)   # [A, P, N, C]
    ref_out = (wc * val).sum(dim=(1, 2))
    god = go[0].double()
    ref_gw = (god[:, None, None, :] * val).reshape(A, P, 2, G, C // G).sum(-1)
    ref_gx = Wd[0, 0][None, None, :] * (wc * god[:, None, None, :] * beta).sum(-1)
    ref_gy = Hd[0, 0][None, None, :] * (wc * god[:, None, None, :] * gamma).sum(-1)
    assert_close(host(out)[0], ref_out.numpy(), FWD_F32_TOL, FWD_F32_MAXREL, "out")
    assert_close(host(gw)[0, :, :, :, 0], ref_gw.numpy(), GRAD_F32_TOL, GRAD_F32_MAXREL, "grad_w")
    assert_close(host(gl)[0, ..., 0], ref_gx.numpy(), GRAD_F32_TOL, GRAD_F32_MAXREL, "grad_loc x")
    assert_close(host(gl)[0, ..., 1], ref_gy.numpy(), GRAD_F32_TOL, GRAD_F32_MAXREL, "grad_loc y")
    # <grad_feat, feat> = <grad_out, out>, in FP64 over row bands
    lhs = 0.0
    for r0 in range(0, R, 1 << 19):
        lhs += float((gf[0, r0:r0 + (1 << 19)].double() * feat[0, r0:r0 + (1 << 19)].double()).sum())
    rhs = float((god * ref_out).sum())
    assert abs(lhs - rhs) <= 1e-5 * (abs(rhs) + 1.0), (lhs, rhs)


def test_bf16_constant_map_beyond_2gib(ops):
    """BF16 storage, one batch item of 2.3 GB (2 cameras x one 2048 x 1100
    level, C = 256): a constant map returns the constant times the sum of the
    weights for samples in the last rows (the highest offsets)."""
    C, G, A, P = 256, 8, 24, 4
    shapes, starts, R = synth.layout([[(2048, 1100)]] * 2)
    assert 2 ** 31 < R * C * 2 <= 2 ** 32 - 8192
    gen = torch.Generator().manual_seed(8)
    feat = torch.full((1, R, C), 1.5, dtype=torch.bfloat16, device="cuda")
    loc = _interior_locs(shapes, A, P, gen)
    w = torch.rand(1, A, P, 2, 1, G, generator=gen)
    layout = ops.Layout(shapes, starts)
    out = ops.forward(feat, layout, loc.cuda(), w.cuda())
    torch.cuda.synchronize()
    ref = 1.5 * w[0, :, :, :, 0].double().sum(dim=(1, 2)).repeat_interleave(C // G, dim=-1)
    assert_close(host(out)[0], ref.numpy(), FWD_F32_TOL, FWD_F32_MAXREL, "constant map")


@pytest.mark.parametrize("which", ["train16", "cam64"])
def test_forward_full_size_sampled(ops, oracle_mod, which):
    """Full-size workloads in the benchmark's launch configuration (default
    tile), FP32 storage; the oracle evaluates a seeded subset of anchors."""
    p = synth.train16() if which == "train16" else synth.cam64()
    print(f"case {p.name} {p.dims()}", flush=True)
    got = run_fwd(ops, p)
    idx = anchor_subset(p, 48, seed=1)
    ref = oracle_forward_subset(oracle_mod, p.feat, p, idx)
    assert_close(got[:, idx], ref, FWD_F32_TOL, FWD_F32_MAXREL, p.name)
    assert np.isfinite(got).all()
