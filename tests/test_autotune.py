"""The launch-shape autotuner: its candidate list matches what the library
accepts, the cache round-trips, and (GPU) tuning picks a shape that
`tile="auto"` then uses."""
import ctypes
import json

import pytest
import torch

from paper_2601_10819_amd import _lib, autotune, synth

FAKE = 0x7f0000000000


def _accepted(lib, dtype_code, C, G, tile):
    shapes = (ctypes.c_int32 * 2)(4, 4)
    starts = (ctypes.c_int32 * 1)(0)
    d = _lib.MsdaDesc()
    d.batch, d.num_cams, d.num_levels, d.num_anchors, d.num_points = 1, 1, 1, 0, 1
    d.channels, d.groups, d.feat_dtype, d.rows = C, G, dtype_code, 16
    d.host_spatial_shapes = ctypes.addressof(shapes)
    d.host_level_start_index = ctypes.addressof(starts)
    d.level_scale = FAKE if dtype_code == _lib.MSDA_FP8_E4M3 else None
    t = _lib.MsdaTile(tile["waves_per_anchor"], tile["chans_per_lane"],
                      _lib.ORDERS[tile.get("order", "auto")], 0)
    d.tile = ctypes.pointer(t)
    # A = 0: validated, nothing launched
    return lib.msda_forward_ws(FAKE, FAKE, FAKE, None, None, None, None, 0, ctypes.byref(d),
                               None) == 0


@pytest.mark.parametrize("dtype,code", [(torch.float32, 0), (torch.bfloat16, 1),
                                        (torch.uint8, 2)])
@pytest.mark.parametrize("C,G", [(256, 8), (64, 4), (128, 8), (32, 2), (96, 3)])
def test_candidates_are_exactly_what_the_library_accepts(dtype, code, C, G):
    lib = _lib.load()
    cands = autotune.candidates(dtype, C, G)
    for t in cands:
        assert _accepted(lib, code, C, G, t), t
    every = [{"waves_per_anchor": w, "chans_per_lane": c, "order": o} for w in (1, 2, 4, 8)
             for c in (1, 2, 4, 8, 16) for o in ("anchor", "view")]
    for t in every:
        if t not in cands:
            assert not _accepted(lib, code, C, G, t), t


def test_shape_key_buckets():
    k1 = autotune.shape_key(torch.bfloat16, 256, 8, 4, 13, 64, 900, arch="gfx950")
    k2 = autotune.shape_key(torch.bfloat16, 256, 8, 4, 13, 60, 1000, arch="gfx950")
    k3 = autotune.shape_key(torch.bfloat16, 256, 8, 4, 13, 64, 1100, arch="gfx950")
    assert k1 == k2 and k1 != k3
    assert autotune.shape_key(torch.float32, 256, 8, 4, 13, 64, 900, arch="gfx950") != k1


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    autotune.save_cache({"a": {"forward": {"waves_per_anchor": 4, "chans_per_lane": 8}}}, path)
    autotune.save_cache({"b": {"tile": {"waves_per_anchor": 2, "chans_per_lane": 4}}}, path)
    data = json.load(open(path))
    assert set(data) == {"a", "b"}
    assert autotune.lookup("a", path)["forward"]["waves_per_anchor"] == 4
    assert autotune.lookup("missing", path) is None
    open(path, "w").write("not json")
    assert autotune.load_cache(path) == {}


@pytest.mark.gpu
def test_tune_single_then_auto(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_10819_amd import ops
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    p = synth.sparse4d(seed=2, anchors=200)
    feat = p.feat.to(torch.bfloat16).cuda()
    layout = ops.Layout(p.spatial_shapes, p.level_start_index)
    loc, w = p.sampling_loc.cuda(), p.weights.cuda()
    go = synth.grad_out_like(p).cuda()
    res = autotune.tune_single(feat, layout, loc, w, go, reps=3)
    assert res["forward"] in autotune.candidates(torch.bfloat16, 256, 8)
    assert res["backward"] in autotune.candidates(torch.bfloat16, 256, 8)
    a = ops.forward(feat, layout, loc, w, tile="auto")
    b = ops.forward(feat, layout, loc, w, tile=res["forward"])
    ga = ops.backward(feat, layout, loc, w, go, tile="auto")
    gb = ops.backward(feat, layout, loc, w, go, tile=res["backward"])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for x, y in zip(ga, gb):
        assert torch.equal(x, y)


@pytest.mark.gpu
def test_tune_batch(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_10819_amd import ops
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    probs = synth.batched(seed=4, scenes=4, scale_anchors=0.05, max_cams=8)
    scenes = [(p.feat[0].to(torch.bfloat16).cuda(), ops.Layout(p.spatial_shapes, p.level_start_index),
               p.sampling_loc[0].cuda(), p.weights[0].cuda()) for p in probs]
    batch = ops.SceneBatch(scenes)
    res = autotune.tune_batch(batch, reps=2)
    assert res["tile"] in autotune.candidates(torch.bfloat16, 256, 8, orders=("anchor", "view"))
    assert batch.tile == res["tile"]
    again = ops.SceneBatch(scenes, tile="auto")
    assert again.tile == res["tile"]
