"""msda_forward_noalloc, the forward for callers that cannot allocate (its
workspace lives in the library's fixed per-GPU scratch array), against
msda_forward_ws with a caller workspace on the same inputs: the outputs must
be bitwise equal (same kernels, same fixed summation order). Calls run back
to back in one process, each over what the previous call left in the
scratch: the 64-camera scene in BF16, then a smaller 16-camera FP32 scene,
then logits weights (the softmax statistics also live in the scratch), and
an input too large for the scratch, which is refused before any launch."""
import ctypes

import pytest
import torch

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


def _case(p, dtype):
    from paper_2601_10819_amd import ops
    feat = p.feat.to(dtype).cuda()
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    return feat, layout, p.sampling_loc.cuda(), p.weights.cuda()


def _check(ops, feat, layout, loc, w, logits=False):
    ref = ops.forward(feat, layout, loc, w, logits=logits)          # msda_forward_ws
    out = torch.full_like(ref, float("nan"))
    ops.forward_noalloc(feat, layout, loc, w, out, logits=logits)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    return out


def test_noalloc_matches_workspace_form(ops):
    big = synth.cam64(seed=0)                               # 64 cameras, 900 anchors
    print(f"noalloc: {big.name} {big.dims()} bf16", flush=True)
    _check(ops, *_case(big, torch.bfloat16))
    small = synth.cam64(seed=3, anchors=200, cams=16)       # smaller, after the big one
    print(f"noalloc: {small.name} {small.dims()} f32", flush=True)
    _check(ops, *_case(small, torch.float32))
    mid = synth.cam64(seed=4, anchors=300, cams=8)
    feat, layout, loc, w = _case(mid, torch.bfloat16)
    g = torch.Generator().manual_seed(6)
    logits = (torch.randn(mid.weights.shape, generator=g) * 2.0).cuda()
    print(f"noalloc: {mid.name} {mid.dims()} bf16 logits", flush=True)
    _check(ops, feat, layout, loc, logits, logits=True)
    # the first workload once more: the leftovers of the others change nothing
    _check(ops, *_case(big, torch.bfloat16))


def test_noalloc_refuses_inputs_beyond_the_scratch(ops):
    lib = ops._lib.load()
    p = synth.cam64(seed=0, anchors=4200, cams=8)           # 8*4200*256*4 B > 32 MiB
    feat, layout, loc, w = _case(p, torch.bfloat16)
    d = ops.make_desc(feat, layout, loc, w)
    assert lib.msda_forward_workspace_size(ctypes.byref(d)) > (32 << 20)
    out = torch.full((1, 4200, 256), 7.0, device="cuda")
    st = lib.msda_forward_noalloc(feat.data_ptr(), layout.shapes.data_ptr(),
                                  layout.starts.data_ptr(), loc.data_ptr(), w.data_ptr(),
                                  out.data_ptr(), ctypes.byref(d), ops._stream())
    torch.cuda.synchronize()
    assert st == ops._lib.MSDA_ERR_UNSUPPORTED
    assert "scratch" in lib.msda_last_error().decode()
    assert bool((out == 7.0).all())                         # nothing was launched
    # the anchor order needs no workspace, so the same input runs
    ref = ops.forward(feat, layout, loc, w, tile={"order": "anchor"})
    got = ops.forward_noalloc(feat, layout, loc, w, torch.empty_like(ref),
                              tile={"order": "anchor"})
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
