"""Batched form: uneven scenes (cameras, resolution, anchors) in one
persistent launch per pass. Checked bit for bit against the single-call
entry points on each scene (same launch shape), against the FP64 oracle,
and under HIP-graph capture and replay."""
import numpy as np
import pytest
import torch

from helpers import (BF16_TOL, FWD_F32_MAXREL, FWD_F32_TOL, GRAD_F32_MAXREL, GRAD_F32_TOL,
                     anchor_subset, assert_close, host, normwise, oracle_backward_subset)
from paper_2601_10819_amd import _lib, synth

pytestmark = pytest.mark.gpu

# single calls compared bit for bit with the batched form run in the same
# work order and lane layout
TILE = {"waves_per_anchor": 4, "order": "anchor"}
VIEW_TILE = {"waves_per_anchor": 2, "order": "view"}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ops():
    from paper_2601_10819_amd import ops as o
    o._lib.load()
    return o


def small_batch(seed=0, scenes=6, scale=0.04, max_cams=6, empty_scene=True):
    probs = synth.batched(seed=seed, scenes=scenes, scale_anchors=scale, max_cams=max_cams)
    if empty_scene:
        p = probs[1]
        probs[1] = synth.Problem(p.name + "_empty", p.feat, p.spatial_shapes, p.level_start_index,
                                 p.sampling_loc[:, :0].contiguous(), p.weights[:, :0].contiguous())
    return probs


def to_scenes(ops, probs, dtype):
    out = []
    for p in probs:
        out.append((p.feat[0].to(dtype).cuda(), ops.Layout(p.spatial_shapes, p.level_start_index),
                    p.sampling_loc[0].cuda(), p.weights[0].cuda()))
    return out


@pytest.mark.parametrize("tile", [TILE, VIEW_TILE], ids=["anchor", "view"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
def test_batched_equals_single_calls_bitwise(ops, dtype, tile):
    """Per scene the batched arithmetic is the single call's in the same
    order (the view order splits each scene over the XCD slots as a single
    call with B = 1 does), so every output is bitwise equal."""
    probs = small_batch(max_cams=11)
    print("case", [p.dims() for p in probs], tile, flush=True)
    scenes = to_scenes(ops, probs, dtype)
    batch = ops.SceneBatch(scenes, tile=tile)
    gen = torch.Generator(device="cuda").manual_seed(5)
    for go in batch.grad_out:
        go.normal_(generator=gen)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    for s, (feat, layout, loc, w) in enumerate(scenes):
        out = ops.forward(feat[None], layout, loc[None], w[None], tile=tile)
        gf, gl, gw = ops.backward(feat[None], layout, loc[None], w[None], batch.grad_out[s][None],
                                  tile=tile)
        torch.cuda.synchronize()
        assert torch.equal(out[0], batch.out[s]), f"scene {s} out"
        assert torch.equal(gf[0], batch.grad_feat[s]), f"scene {s} grad_feat"
        assert torch.equal(gl[0], batch.grad_loc[s]), f"scene {s} grad_loc"
        assert torch.equal(gw[0], batch.grad_w[s]), f"scene {s} grad_w"


def test_batched_matches_oracle(ops, oracle_mod):
    probs = small_batch(seed=1, scenes=4, scale=0.02, max_cams=4)
    scenes = to_scenes(ops, probs, torch.float32)
    batch = ops.SceneBatch(scenes)
    gos = [synth.grad_out_like(p, seed=10 + s)[0] for s, p in enumerate(probs)]
    for go, g in zip(batch.grad_out, gos):
        go.copy_(g)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    for s, p in enumerate(probs):
        if p.num_anchors == 0:
            assert batch.out[s].numel() == 0
            assert torch.all(batch.grad_feat[s] == 0)
            continue
        ref = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                                 p.weights)
        assert_close(host(batch.out[s])[None], ref, FWD_F32_TOL, FWD_F32_MAXREL, f"scene {s} out")
        rgf, rgl, rgw = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index,
                                            p.sampling_loc, p.weights, gos[s][None])
        assert_close(host(batch.grad_feat[s])[None], rgf, GRAD_F32_TOL, GRAD_F32_MAXREL, "gf")
        assert_close(host(batch.grad_loc[s])[None], rgl, GRAD_F32_TOL, GRAD_F32_MAXREL, "gl")
        assert_close(host(batch.grad_w[s])[None], rgw, GRAD_F32_TOL, GRAD_F32_MAXREL, "gw")


def test_batched_graph_capture_replay(ops):
    """Forward + backward captured once and replayed: every replay equals the
    eager result bit for bit, with eager work and synchronisation between
    replays; an input updated in place between replays is picked up."""
    probs = small_batch(seed=2, scenes=5, scale=0.03, max_cams=5)
    scenes = to_scenes(ops, probs, torch.bfloat16)
    batch = ops.SceneBatch(scenes)
    gen = torch.Generator(device="cuda").manual_seed(6)
    for go in batch.grad_out:
        go.normal_(generator=gen)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    eager = [t.clone() for t in batch.out + batch.grad_feat + batch.grad_loc + batch.grad_w]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            batch.forward()
            batch.backward()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in batch.out + batch.grad_feat + batch.grad_loc + batch.grad_w:
            t.fill_(float("nan") if t.is_floating_point() else 0)   # eager work in between
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        now = batch.out + batch.grad_feat + batch.grad_loc + batch.grad_w
        for a, b in zip(now, eager):
            assert torch.equal(a, b), f"replay {rep}"
    # update one scene's weights in place: the replay uses the new values
    scenes[0][3].mul_(2.0)
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(batch.out[0], eager[0] * 2.0)


def test_batched_full_size_bf16(ops, oracle_mod):
    """The 12-scene uneven batch at full size (BF16 features): a sampled
    check against the oracle per scene and the Euler identity per scene."""
    probs = synth.batched(seed=0)
    print("scenes", [(p.num_cams, p.rows, p.num_anchors) for p in probs], flush=True)
    scenes = to_scenes(ops, probs, torch.bfloat16)
    batch = ops.SceneBatch(scenes)
    gen = torch.Generator(device="cuda").manual_seed(7)
    for go in batch.grad_out:
        go.normal_(generator=gen)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    for s in (0, 5, 11):
        p = probs[s]
        idx = anchor_subset(p, 8, seed=s)
        feat64 = p.feat.to(torch.bfloat16).double()
        ref = oracle_mod.forward(feat64, p.spatial_shapes, p.level_start_index,
                                 p.sampling_loc[:, idx].contiguous(), p.weights[:, idx].contiguous())
        assert_close(host(batch.out[s])[idx][None], ref, FWD_F32_TOL, FWD_F32_MAXREL, f"scene {s}")
        # grad_sampling_loc and grad_weights of the same anchors (per-anchor
        # quantities) against the oracle's analytic gradient
        go = batch.grad_out[s].cpu()[None]
        rgl, rgw = oracle_backward_subset(oracle_mod, feat64, p, idx, go)
        assert_close(host(batch.grad_loc[s])[idx][None], rgl, GRAD_F32_TOL, GRAD_F32_MAXREL,
                     f"scene {s} grad_loc")
        assert_close(host(batch.grad_w[s])[idx][None], rgw, GRAD_F32_TOL, GRAD_F32_MAXREL,
                     f"scene {s} grad_w")
    for s in range(len(probs)):
        feat, layout, loc, w = scenes[s]
        e_out = float((batch.out[s].double() * batch.grad_out[s].double()).sum())
        pf = batch.grad_feat[s].double() * feat.double()
        pw = batch.grad_w[s].double() * w.double()
        # grad_feat is rounded to BF16 once per element (relative error <= 2^-9
        # each), so the identity holds to 2^-9 of the sum of |terms|
        assert abs(float(pf.sum()) - e_out) <= 2.0 ** -9 * float(pf.abs().sum()), (s, e_out)
        assert abs(float(pw.sum()) - e_out) <= 1e-5 * float(pw.abs().sum()), (s, e_out)


def test_batched_single_scene_and_validation(ops):
    probs = small_batch(seed=3, scenes=1, empty_scene=False)
    scenes = to_scenes(ops, probs, torch.float32)
    batch = ops.SceneBatch(scenes, tile=TILE)
    batch.forward()
    torch.cuda.synchronize()
    feat, layout, loc, w = scenes[0]
    out = ops.forward(feat[None], layout, loc[None], w[None], tile=TILE)
    torch.cuda.synchronize()
    assert torch.equal(out[0], batch.out[0])
    # mixed gradient requests are rejected
    with pytest.raises(ValueError):
        ops.SceneBatch(scenes + [(feat.to(torch.bfloat16), layout, loc, w)])


def test_batched_view_order_tiny_scenes(ops):
    """Scenes with fewer (camera, anchor) items than XCD slots leave slots
    empty (their rows add zeros): the view-order batch still equals the
    single calls in view order on every scene, bit for bit."""
    probs = [synth.small(seed=60, cams=1, A=3, P=3, C=64, G=4),
             synth.small(seed=61, cams=2, A=1, P=3, C=64, G=4),
             synth.small(seed=62, cams=5, A=9, P=3, C=64, G=4),
             synth.small(seed=63, cams=13, A=2, P=3, C=64, G=4)]
    print("case", [p.dims() for p in probs], flush=True)
    scenes = to_scenes(ops, probs, torch.float32)
    batch = ops.SceneBatch(scenes, tile=VIEW_TILE)
    gen = torch.Generator(device="cuda").manual_seed(7)
    for go in batch.grad_out:
        go.normal_(generator=gen)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    for s, (feat, layout, loc, w) in enumerate(scenes):
        out = ops.forward(feat[None], layout, loc[None], w[None], tile=VIEW_TILE)
        gf, gl, gw = ops.backward(feat[None], layout, loc[None], w[None], batch.grad_out[s][None],
                                  tile=VIEW_TILE)
        torch.cuda.synchronize()
        assert torch.equal(out[0], batch.out[s]), f"scene {s} out"
        assert torch.equal(gf[0], batch.grad_feat[s]), f"scene {s} grad_feat"
        assert torch.equal(gl[0], batch.grad_loc[s]), f"scene {s} grad_loc"
        assert torch.equal(gw[0], batch.grad_w[s]), f"scene {s} grad_w"


@pytest.mark.parametrize("big", ["anchors", "level"])
def test_batched_record_sort_forms_bitwise(ops, big):
    """The batched grad_feat records are sorted per (scene, region) bucket
    when every scene's A*P fits one bucket-sort block (at most 2^15) and
    every region's cells its keys (at most 2^17), else by the global radix
    sort over the whole batch. Either way each cell's records end in sample
    order: a batch with one scene beyond a limit (A*P = 33000, or a
    400 x 400 level) still equals the single calls bit for bit, and so does
    the same batch without that scene (bucketed)."""
    if big == "anchors":
        large = synth.small(seed=70, cams=2, A=11000, P=3, C=32, G=4,
                            levels=((20, 30), (10, 15)))
    else:
        large = synth.small(seed=70, cams=2, A=40, P=3, C=32, G=4,
                            levels=((400, 400), (10, 15)))
    rest = [synth.small(seed=71, cams=3, A=7, P=3, C=32, G=4, levels=((12, 9), (6, 5))),
            synth.small(seed=72, cams=1, A=1, P=3, C=32, G=4, levels=((3, 4), (2, 2)))]
    for probs in ([large] + rest, rest):
        print("case", big, [p.dims() for p in probs], flush=True)
        scenes = to_scenes(ops, probs, torch.float32)
        batch = ops.SceneBatch(scenes, tile=VIEW_TILE)
        gen = torch.Generator(device="cuda").manual_seed(8)
        for go in batch.grad_out:
            go.normal_(generator=gen)
        batch.forward()
        batch.backward()
        torch.cuda.synchronize()
        for s, (feat, layout, loc, w) in enumerate(scenes):
            gf, gl, gw = ops.backward(feat[None], layout, loc[None], w[None],
                                      batch.grad_out[s][None], tile=VIEW_TILE)
            torch.cuda.synchronize()
            assert torch.equal(gf[0], batch.grad_feat[s]), f"scene {s} grad_feat"
            assert torch.equal(gl[0], batch.grad_loc[s]), f"scene {s} grad_loc"
            assert torch.equal(gw[0], batch.grad_w[s]), f"scene {s} grad_w"


def test_batched_global_sort_on_request_bitwise(ops):
    """MSDA_SCATTER_SORTED_GLOBAL sends the batch's records through the
    global radix sort instead of the per-(scene, region) buckets: every
    output bitwise the same (BF16, view order, one scene without anchors)."""
    probs = small_batch(seed=11, scenes=5, max_cams=9)
    print("case", [p.dims() for p in probs], flush=True)
    scenes = to_scenes(ops, probs, torch.bfloat16)
    res = []
    for scatter in (0, _lib.MSDA_SCATTER_SORTED_GLOBAL):
        batch = ops.SceneBatch(scenes, tile=dict(VIEW_TILE, scatter=scatter))
        gen = torch.Generator(device="cuda").manual_seed(12)
        for go in batch.grad_out:
            go.normal_(generator=gen)
        batch.forward()
        batch.backward()
        torch.cuda.synchronize()
        res.append(batch)
    a, b = res
    for s in range(len(scenes)):
        assert torch.equal(a.grad_feat[s], b.grad_feat[s]), f"scene {s} grad_feat"
        assert torch.equal(a.grad_loc[s], b.grad_loc[s]), f"scene {s} grad_loc"
        assert torch.equal(a.grad_w[s], b.grad_w[s]), f"scene {s} grad_w"


@pytest.mark.parametrize("tile", [TILE, VIEW_TILE], ids=["anchor", "view"])
@pytest.mark.parametrize("wkind", ["logits_f32", "logits_bf16", "weights_bf16"])
def test_batched_weight_flags_equal_single_calls(ops, wkind, tile):
    """Weight flags in the batched form: per-group softmax of logits (FP32 or
    BF16), or BF16 weights. Per scene the statistics, the FP32 weights of the
    backward and the gradient through the softmax are the single call's, so
    every output is bitwise equal to per-scene calls with the same flag (one
    scene has no anchors)."""
    probs = small_batch(seed=9, scenes=5, max_cams=9)
    logits = wkind.startswith("logits")
    wdt = torch.float32 if wkind == "logits_f32" else torch.bfloat16
    print("case", wkind, tile, [p.dims() for p in probs], flush=True)
    scenes = [(f, lay, loc, (w * 3.0 if logits else w).to(wdt).contiguous())
              for f, lay, loc, w in to_scenes(ops, probs, torch.bfloat16)]
    batch = ops.SceneBatch(scenes, tile=tile, logits=logits)
    gen = torch.Generator(device="cuda").manual_seed(10)
    for go in batch.grad_out:
        go.normal_(generator=gen)
    batch.forward()
    batch.backward()
    torch.cuda.synchronize()
    for s, (feat, layout, loc, w) in enumerate(scenes):
        out = ops.forward(feat[None], layout, loc[None], w[None], tile=tile, logits=logits)
        gf, gl, gw = ops.backward(feat[None], layout, loc[None], w[None], batch.grad_out[s][None],
                                  tile=tile, logits=logits)
        torch.cuda.synchronize()
        assert torch.equal(out[0], batch.out[s]), f"scene {s} out"
        assert torch.equal(gf[0], batch.grad_feat[s]), f"scene {s} grad_feat"
        assert torch.equal(gl[0], batch.grad_loc[s]), f"scene {s} grad_loc"
        assert torch.equal(gw[0], batch.grad_w[s]), f"scene {s} grad_w"


def test_batched_rejects_uneven_shared_sizes(ops):
    """Keypoints, levels, channels and groups are shared by a batch: a scene
    that differs is rejected before anything runs."""
    base = small_batch(seed=3, scenes=2, empty_scene=False)
    odd = synth.small(seed=64, cams=3, A=4, P=base[0].num_points + 1, C=base[0].channels,
                      G=base[0].groups, levels=((6, 10), (3, 5), (2, 3), (1, 2)))
    scenes = to_scenes(ops, base + [odd], torch.float32)
    with pytest.raises(ValueError, match="sampling_loc"):
        ops.SceneBatch(scenes)
