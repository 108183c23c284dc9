"""Precision forms: BF16, FP16 and FP8-e4m3 feature storage with FP32
arithmetic.

Each is measured two ways against the FP64 oracle: the kernel error (oracle
run on the stored values, widened exactly) must meet the FP32 bar, and the
total error (oracle run on the original FP32 features) is reported, with the
half-precision bar of 1e-2 of the output RMS (FP16, with 3 more mantissa
bits than BF16, is also held to 1e-3)."""
import numpy as np
import pytest
import torch

from helpers import (BF16_TOL, FWD_F32_MAXREL, FWD_F32_TOL, GRAD_F32_TOL, anchor_subset,
                     assert_close, host, normwise, oracle_backward_subset,
                     oracle_forward_subset, to_device)
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


HALF = [torch.bfloat16, torch.float16]
HALF_IDS = ["bf16", "f16"]
# total-error bar per storage type, and the bar on grad_feat against the
# oracle's sum rounded to that type (the rounding differs by at most one
# ulp where the FP32 and FP64 sums straddle a rounding boundary)
TOTAL_TOL = {torch.bfloat16: BF16_TOL, torch.float16: 1e-3}
ROUNDED_TOL = {torch.bfloat16: 5e-3, torch.float16: 5e-4}


def widened(p, dtype):
    return p.feat.to(dtype).double()


@pytest.mark.parametrize("dtype", HALF, ids=HALF_IDS)
@pytest.mark.parametrize("which", ["sparse4d", "train16", "cam64"])
def test_half_forward(ops, oracle_mod, which, dtype):
    p = {"sparse4d": lambda: synth.sparse4d(seed=0), "train16": synth.train16,
         "cam64": synth.cam64}[which]()
    feat, layout, loc, w = to_device(p, dtype)
    got = host(ops.forward(feat, layout, loc, w))
    idx = anchor_subset(p, 64, seed=3)
    ref_kernel = oracle_forward_subset(oracle_mod, widened(p, dtype), p, idx)
    ref_total = oracle_forward_subset(oracle_mod, p.feat, p, idx)
    assert_close(got[:, idx], ref_kernel, FWD_F32_TOL, FWD_F32_MAXREL, f"{which} {dtype} kernel")
    total = normwise(got[:, idx], ref_total)
    print(f"{which} {dtype} forward total error {total:.3e}", flush=True)
    assert total <= TOTAL_TOL[dtype]


@pytest.mark.parametrize("dtype", HALF, ids=HALF_IDS)
@pytest.mark.parametrize("which", ["sparse4d", "train16", "cam64"])
def test_half_backward(ops, oracle_mod, which, dtype):
    """Every gradient through the library's default backward (view order at
    16 and 64 cameras, the 3-pass record sort, the tile reduction's BF16 /
    FP16 store): grad_loc and grad_w on an anchor subset, grad_feat in full,
    each against the oracle on the stored (widened) features and on the
    original FP32 features."""
    p = {"sparse4d": lambda: synth.sparse4d(seed=0), "train16": synth.train16,
         "cam64": synth.cam64}[which]()
    print(f"case {p.name} {p.dims()} {dtype}", flush=True)
    go = synth.grad_out_like(p, seed=7)
    feat, layout, loc, w = to_device(p, dtype)
    gf, gl, gw = ops.backward(feat, layout, loc, w, go.cuda())
    torch.cuda.synchronize()
    assert gf.dtype == dtype
    idx = anchor_subset(p, 48, seed=4)
    rgl_k, rgw_k = oracle_backward_subset(oracle_mod, widened(p, dtype), p, idx, go)
    rgl_t, rgw_t = oracle_backward_subset(oracle_mod, p.feat, p, idx, go)
    assert_close(host(gl)[:, idx], rgl_k, GRAD_F32_TOL, None, f"{which} {dtype} grad_loc kernel")
    assert_close(host(gw)[:, idx], rgw_k, GRAD_F32_TOL, None, f"{which} {dtype} grad_w kernel")
    assert normwise(host(gl)[:, idx], rgl_t) <= TOTAL_TOL[dtype]
    assert normwise(host(gw)[:, idx], rgw_t) <= TOTAL_TOL[dtype]
    rgf, _, _ = oracle_mod.backward(widened(p, dtype), p.spatial_shapes, p.level_start_index,
                                    p.sampling_loc, p.weights, go, need_loc=False, need_w=False)
    # grad_feat is rounded once to the storage type: error bounded by the
    # type's bar, and the rounding is to nearest (within half an ulp of the
    # FP32 sum, so at most one ulp from the oracle's sum rounded the same way)
    err = normwise(host(gf), rgf)
    print(f"{which} {dtype} grad_feat error {err:.3e}", flush=True)
    assert err <= TOTAL_TOL[dtype]
    rounded = torch.from_numpy(rgf).float().to(dtype).double().numpy()
    assert normwise(host(gf), rounded) <= ROUNDED_TOL[dtype]
    # elements the oracle sum leaves far from a rounding boundary round the
    # same way: the FP32 sum differs from the FP64 one by far less than the
    # spacing of the storage type
    assert np.mean(host(gf) == rounded) >= 0.99


def test_f16_grad_feat_rounding_is_ieee(ops):
    """Pixel-centre samples with one weight each: grad_feat is w * grad_out
    summed in FP32 and rounded once to IEEE half (nearest even), overflow to
    infinity included."""
    C, G = 64, 4
    shapes, starts, R = synth.layout([[(1, 4)]])
    layout = ops.Layout(shapes, starts)
    feat = torch.zeros(1, R, C, dtype=torch.float16, device="cuda")
    A = 4
    loc = torch.zeros(1, A, 1, 1, 2)
    loc[0, :, 0, 0, 0] = (torch.arange(A) + 0.5) / 4      # pixel a of the 1x4 level
    loc[0, :, 0, 0, 1] = 0.5
    w = torch.ones(1, A, 1, 1, 1, G)
    go = torch.randn(1, A, C, generator=torch.Generator().manual_seed(0)) * 3.0
    go[0, 3, :8] = torch.tensor([7e4, -7e4, 65504.0, 65519.0, 65520.0, 1e-8, 3e-5, 6.1e-5])
    gf, _, _ = ops.backward(feat, layout, loc.cuda(), w.cuda(), go.cuda(), need_loc=False,
                            need_w=False)
    torch.cuda.synchronize()
    want = go[0].to(torch.float16)                          # torch's FP32 -> half (RNE)
    assert torch.equal(gf[0, :A].cpu(), want)


@pytest.mark.parametrize("C", [64, 256])
def test_bf16_grad_feat_rounding_is_rne(ops, C):
    """Pixel-centre samples with one weight each: grad_feat is w * grad_out
    rounded once to bfloat16, nearest even, against torch's FP32 -> bfloat16
    cast: exact ties both ways, the largest finite values and overflow,
    FP32 subnormals, zeros of both signs, and random values. C = 64 runs the tile
    reduction with 16 lanes per pixel, C = 256 with whole waves."""
    G = 4
    shapes, starts, R = synth.layout([[(1, 4)]])
    layout = ops.Layout(shapes, starts)
    feat = torch.zeros(1, R, C, dtype=torch.bfloat16, device="cuda")
    A = 4
    loc = torch.zeros(1, A, 1, 1, 2)
    loc[0, :, 0, 0, 0] = (torch.arange(A) + 0.5) / 4      # pixel a of the 1x4 level
    loc[0, :, 0, 0, 1] = 0.5
    w = torch.ones(1, A, 1, 1, 1, G)
    go = torch.randn(1, A, C, generator=torch.Generator().manual_seed(0)) * 3.0
    one = 1.0
    tie_even = one + 2.0 ** -8            # halfway between 1 and 1 + 2^-7: rounds down
    tie_odd = one + 3 * 2.0 ** -8         # halfway, odd below: rounds up
    special = torch.tensor([tie_even, tie_odd, -tie_even, -tie_odd, 3.3895e38, 3.4e38,
                            -3.4e38, 1e-40, -1e-40, 2.0 ** -133, 0.0, -0.0,
                            1.0 + 2.0 ** -8 + 2.0 ** -20, 2.0 ** -126, 65504.0, 1e-8],
                           dtype=torch.float32)
    go[0, 3, :len(special)] = special
    gf, _, _ = ops.backward(feat, layout, loc.cuda(), w.cuda(), go.cuda(), need_loc=False,
                            need_w=False)
    torch.cuda.synchronize()
    # the FP32 sum starts at +0 (so -0 sums to +0), then torch's FP32 ->
    # bfloat16 cast (nearest even)
    want = (go[0] + 0.0).to(torch.bfloat16)
    got = gf[0, :A].cpu()
    assert torch.equal(got.view(torch.int16), want.view(torch.int16)), \
        [(float(go[0].reshape(-1)[i]), int(got.view(torch.int16).reshape(-1)[i]),
          int(want.view(torch.int16).reshape(-1)[i]))
         for i in torch.nonzero(got.view(torch.int16).reshape(-1) !=
                                want.view(torch.int16).reshape(-1)).reshape(-1)[:8]]


def test_fp8_quantiser_bit_exact(ops, oracle_mod):
    p = synth.sparse4d(seed=1, anchors=8)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    codes, scales = ops.quantize_fp8(p.feat.cuda(), layout)
    torch.cuda.synchronize()
    rcodes, rscales = oracle_mod.quantize_fp8_per_level(p.feat, p.spatial_shapes,
                                                         p.level_start_index)
    assert np.array_equal(scales.cpu().numpy(), rscales)
    assert np.array_equal(codes.cpu().numpy(), rcodes)


def test_fp8_quantiser_bit_exact_cam64(ops, oracle_mod):
    """The benchmarked 64-camera pyramid (64 x 4 regions, C = 256): the
    vector path over regions of 8 to 7,168 rows, bit-exact."""
    p = synth.cam64(seed=0, anchors=1)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    codes, scales = ops.quantize_fp8(p.feat.cuda(), layout)
    torch.cuda.synchronize()
    rcodes, rscales = oracle_mod.quantize_fp8_per_level(p.feat, p.spatial_shapes,
                                                         p.level_start_index)
    assert np.array_equal(scales.cpu().numpy(), rscales)
    assert np.array_equal(codes.cpu().numpy(), rcodes)


def test_fp8_quantiser_rounding_boundaries(ops, oracle_mod):
    """The encoder's rounding at every boundary of the format. A level whose
    largest |x| is 448 has scale 1, so each value reaches the encoder
    unchanged: every finite e4m3 value, every midpoint between neighbours
    (ties go to the even code), the FP32 neighbours of each midpoint, both
    signs, and tiny values below the smallest subnormal (2^-9)."""
    pos = np.sort(oracle_mod.decode_e4m3(np.arange(0, 0x7F, dtype=np.uint8))).astype(np.float32)
    mids = ((pos[:-1].astype(np.float64) + pos[1:]) / 2).astype(np.float32)
    vals = np.concatenate([pos, mids, np.nextafter(mids, np.float32(np.inf)),
                           np.nextafter(mids, np.float32(0)),
                           np.float32([1e-30, 2.0 ** -11, 2.0 ** -10, 3 * 2.0 ** -11, 448.0])])
    vals = np.concatenate([vals, -vals]).astype(np.float32)
    C = 64
    rows = (len(vals) + C - 1) // C
    flat = np.zeros(rows * C, dtype=np.float32)
    flat[:len(vals)] = vals
    feat = torch.from_numpy(flat.reshape(1, rows, C).copy())
    shapes = torch.tensor([[[1, rows]]], dtype=torch.int32)
    starts = torch.zeros(1, 1, dtype=torch.int32)
    layout = ops.Layout(shapes, starts)
    codes, scales = ops.quantize_fp8(feat.cuda(), layout)
    torch.cuda.synchronize()
    assert float(scales[0]) == 1.0
    rcodes, rscales = oracle_mod.quantize_fp8_per_level(feat, shapes, starts)
    assert rscales[0] == 1.0
    got, want = codes.cpu().numpy().reshape(-1), rcodes.reshape(-1)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(float(flat[i]), int(got[i]), int(want[i])) for i in bad[:8]]


@pytest.mark.parametrize("C", [6, 20, 256])
def test_fp8_quantiser_ragged(ops, oracle_mod, C):
    """Two batch items, regions in a permuted order with unused rows between
    them (their codes must be 0), a level whose values are all zero (scale
    1), values far beyond 448 x scale in one level, and C = 6 (the scalar
    path) beside C = 20 and 256 (the vector path)."""
    shapes = torch.tensor([[[5, 7], [3, 4], [1, 1]], [[2, 9], [4, 4], [1, 1]]], dtype=torch.int32)
    starts = torch.tensor([[20, 3, 90], [100, 60, 80]], dtype=torch.int32)
    R = 130
    g = torch.Generator().manual_seed(5)
    feat = torch.randn(2, R, C, generator=g)
    feat[:, 90] = 0.0
    feat[:, 80] = 0.0                                      # level 2 all zero
    feat[1, 61, :3] = torch.tensor([3e4, -5e-7, 1e-30])    # level 1: wide range
    layout = ops.Layout(shapes, starts)
    dev = feat.cuda()
    codes, scales = ops.quantize_fp8(dev, layout)
    torch.cuda.synchronize()
    rcodes, rscales = oracle_mod.quantize_fp8_per_level(feat, shapes, starts)
    assert rscales[2] == 1.0
    assert np.array_equal(scales.cpu().numpy(), rscales)
    assert np.array_equal(codes.cpu().numpy(), rcodes)
    # codes of unused rows are zero even over a buffer that held other bytes
    codes2 = torch.full_like(codes, 0x5A)
    lib = ops._lib.load()
    d = ops._lib.MsdaDesc()
    d.batch, d.num_cams, d.num_levels = 2, 2, 3
    d.num_anchors, d.num_points, d.channels, d.groups = 0, 1, C, 1
    d.feat_dtype, d.rows = ops._lib.MSDA_F32, R
    d.host_spatial_shapes = layout.host_shapes.ctypes.data
    d.host_level_start_index = layout.host_starts.ctypes.data
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    sc2 = torch.empty(3, dtype=torch.float32, device="cuda")
    import ctypes
    ops._lib.check(lib.msda_quantize_fp8(dev.data_ptr(), layout.shapes.data_ptr(),
                                         layout.starts.data_ptr(), codes2.data_ptr(),
                                         sc2.data_ptr(), ws.data_ptr(), ws.numel(),
                                         ctypes.byref(d), ops._stream()))
    torch.cuda.synchronize()
    assert np.array_equal(codes2.cpu().numpy(), rcodes)


def test_fp8_decode_all_codes(ops, oracle_mod):
    """Every e4m3 code through the forward kernel at exact pixel centres
    (one channel group per code byte): out = decode(code) * scale exactly."""
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    C, G = 64, 4
    ncode = len(codes)                            # 254 codes -> 4 rows x 64 channels
    rows_needed = (ncode + C - 1) // C
    levels = [(1, 4)]
    shapes, starts, R = synth.layout([levels])
    assert R >= rows_needed
    table = np.zeros((1, R, C), dtype=np.uint8)
    table.reshape(-1)[:ncode] = codes
    A = R
    loc = torch.zeros(1, A, 1, 1, 2)
    loc[0, :, 0, 0, 0] = (torch.arange(A) + 0.5) / 4
    loc[0, :, 0, 0, 1] = 0.5
    w = torch.ones(1, A, 1, 1, 1, G)
    scale = torch.tensor([0.5], dtype=torch.float32)
    layout = ops.Layout(shapes, starts)
    out = ops.forward(torch.from_numpy(table).cuda(), layout, loc.cuda(), w.cuda(),
                      level_scale=scale.cuda())
    torch.cuda.synchronize()
    got = out.cpu().double().numpy().reshape(-1)[:ncode]
    want = oracle_mod.decode_e4m3(codes) * 0.5
    assert np.array_equal(got, want)


@pytest.mark.parametrize("which", ["sparse4d", "cam64"])
def test_fp8_forward(ops, oracle_mod, which):
    p = synth.sparse4d(seed=0) if which == "sparse4d" else synth.cam64()
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    codes, scales = ops.quantize_fp8(p.feat.cuda(), layout)
    loc, w = p.sampling_loc.cuda(), p.weights.cuda()
    got = host(ops.forward(codes, layout, loc, w, level_scale=scales))
    idx = anchor_subset(p, 48, seed=5)
    deq = oracle_mod.dequantize_fp8(codes.cpu().numpy(), scales.cpu().numpy(), p.spatial_shapes,
                                    p.level_start_index)
    ref_kernel = oracle_forward_subset(oracle_mod, deq, p, idx)
    assert_close(got[:, idx], ref_kernel, FWD_F32_TOL, FWD_F32_MAXREL, f"{which} fp8 kernel")
    ref_total = oracle_forward_subset(oracle_mod, p.feat, p, idx)
    total = normwise(got[:, idx], ref_total)
    print(f"{which} fp8 forward total error {total:.3e}", flush=True)
    # e4m3 keeps 3 mantissa bits: a few percent per element, averaged by the
    # aggregation; a loose sanity bound (the number itself is reported)
    assert total <= 0.1


def test_fp8_backward_rejected(ops):
    p = synth.small(seed=1, C=64, G=4)
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    codes, scales = ops.quantize_fp8(p.feat.cuda(), layout)
    with pytest.raises(ops._lib.MSDAError, match="UNSUPPORTED"):
        ops.backward(codes, layout, p.sampling_loc.cuda(), p.weights.cuda(),
                     torch.zeros(1, p.num_anchors, 64, device="cuda"), level_scale=scales)
