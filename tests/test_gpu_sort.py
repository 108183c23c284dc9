"""The record sort of the deterministic grad_feat reduction (samples' records
grouped by bilinear cell), through its own entry point: bit-exact against
numpy's stable argsort and searchsorted, over one to four radix passes (keys
of 1 to 29 bits), ragged tiles, heavy duplicates and already ordered inputs."""
import numpy as np
import pytest
import torch

from paper_2601_10819_amd import ops

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (n, max_key, key recipe)
CASES = [
    (0, 10, "uniform"),
    (1, 0, "uniform"),
    (4095, 7, "uniform"),              # under one tile, one 3-bit pass
    (4097, 1023, "uniform"),           # ragged second tile, one 10-bit pass
    (300_000, 1024, "uniform"),        # 11-bit keys: two 6-bit passes
    (70_001, 630_000, "uniform"),      # 20-bit keys (the 64-camera cell space): three 7-bit passes
    (200_000, 630_000, "sentinel"),    # most records outside their level (sentinel key)
    (100_000, 630_000, "sorted"),
    (100_000, 630_000, "reversed"),
    (65_536, 630_000, "clustered"),    # runs of equal keys longer than a tile
    (50_000, (1 << 24) - 1, "uniform"),  # three 8-bit passes
    (100_000, (1 << 25) - 1, "uniform"),  # 25-bit keys: four 7-bit passes
    (30_000, (1 << 28) + 12_345, "sentinel"),  # 29-bit keys: four 8-bit passes
    (2_995_200, 630_000, "uniform"),   # the 64-camera scene's record count: 732 tiles, 23 bands
    (20_056_660, 4_000_000, "sentinel"),  # the 12-scene batch's: 4,897 tiles, 154 bands
]


def make_keys(n, max_key, recipe, seed):
    rng = np.random.default_rng(seed)
    if recipe == "uniform":
        return rng.integers(0, max_key + 1, size=n, dtype=np.int64)
    if recipe == "sentinel":
        k = rng.integers(0, max_key, size=n, dtype=np.int64)
        k[rng.random(n) < 0.7] = max_key
        return k
    if recipe == "sorted":
        return np.sort(rng.integers(0, max_key + 1, size=n, dtype=np.int64))
    if recipe == "reversed":
        return np.sort(rng.integers(0, max_key + 1, size=n, dtype=np.int64))[::-1].copy()
    if recipe == "clustered":
        return np.repeat(rng.integers(0, max_key + 1, size=n // 8192 + 1), 8192)[:n]
    raise ValueError(recipe)


@pytest.mark.parametrize("n,max_key,recipe", CASES)
def test_sort_matches_stable_argsort(n, max_key, recipe):
    print(f"sort n={n} max_key={max_key} {recipe}", flush=True)
    keys = make_keys(n, max_key, recipe, seed=n + 7 * max_key)
    k_dev = torch.from_numpy(keys.astype(np.int32)).to(DEV)
    order, seg = ops.sort_keys(k_dev, max_key)
    torch.cuda.synchronize()
    ref = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(order.cpu().numpy(), ref)
    ref_seg = np.searchsorted(keys[ref], np.arange(max_key + 1), side="left")
    np.testing.assert_array_equal(seg.cpu().numpy(), ref_seg)


def test_two_sizes_back_to_back():
    # a second, smaller sort right after a larger one
    for n, seed in ((150_000, 1), (9_000, 2)):
        keys = make_keys(n, 630_000, "uniform", seed)
        order, seg = ops.sort_keys(torch.from_numpy(keys.astype(np.int32)).to(DEV), 630_000)
        np.testing.assert_array_equal(order.cpu().numpy(), np.argsort(keys, kind="stable"))


def test_kernel_event_filter_records_only_the_named_kernel():
    # the benchmark times its roofline kernel this way: with the filter set,
    # only that kernel's launches take event slots (three radix passes here)
    import ctypes

    from bench import HipEvents
    from paper_2601_10819_amd import _lib

    lib = _lib.load()
    ev = HipEvents()
    cap = 8
    arr = (ctypes.c_void_p * (2 * cap))(*[ev.create() for _ in range(2 * cap)])
    keys = torch.from_numpy(make_keys(100_000, 630_000, "uniform", 3).astype(np.int32)).to(DEV)
    try:
        assert lib.msda_set_kernel_event_filter(b"radix_scatter") == _lib.MSDA_OK
        assert lib.msda_set_kernel_events(arr, cap) == _lib.MSDA_OK
        ops.sort_keys(keys, 630_000)
        names = [lib.msda_recorded_kernel_name(i).decode()
                 for i in range(lib.msda_recorded_kernels())]
        lib.msda_set_kernel_events(None, 0)
        torch.cuda.synchronize()
        assert names == ["radix_scatter"] * 3
        assert all(ev.elapsed_ms(arr[2 * i], arr[2 * i + 1]) > 0 for i in range(3))
        # without the filter every launch of the sort is recorded
        assert lib.msda_set_kernel_event_filter(None) == _lib.MSDA_OK
        assert lib.msda_set_kernel_events(arr, cap) == _lib.MSDA_OK
        ops.sort_keys(keys, 630_000)
        n_all = lib.msda_recorded_kernels()
        lib.msda_set_kernel_events(None, 0)
        torch.cuda.synchronize()
        assert n_all == min(cap, 3 * 4 + 1)
    finally:
        lib.msda_set_kernel_events(None, 0)
        lib.msda_set_kernel_event_filter(None)
        for e in arr:
            ev.destroy(e)
