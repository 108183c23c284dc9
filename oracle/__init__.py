"""FP64 CPU oracle for multi-scale deformable aggregation (MSDA).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library
and its Python binding) never does, and the two share no code.

The arithmetic lives in ``msda_oracle.c`` (plain loops in double precision,
OpenMP over independent outputs). This module builds it with gcc, loads it with
ctypes and adds the FP8 helpers of the precision form:

* ``forward`` / ``backward``: MSDA and its analytic gradient (paper Sec. 3.1,
  Sec. 3.2; operator named in Sec. 5.3);
* ``decode_e4m3`` / ``encode_e4m3``: OCP FP8 E4M3 (e4m3fn) by its definition;
* ``quantize_fp8_per_level``: per-level symmetric quantisation,
  scale_l = amax_l / 448, code = RNE(clamp(x / scale_l, +-448));
* ``dequantize_fp8``: code * scale_l, exact in double.

Parity status: forward, backward, encode and decode are pinned by the CPU tests
(closed forms, grid_sample, finite differences, identities, torch's FP8 type).
Agreement with the paper's own (unpublished) kernel is parity unpinned: the
paper prints no MSDA values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msda_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        lib.msda_oracle_forward.argtypes = [i32] * 7 + [i64] + [vp] * 6 + [i32]
        lib.msda_oracle_forward.restype = None
        lib.msda_oracle_backward.argtypes = [i32] * 7 + [i64] + [vp] * 9 + [i32]
        lib.msda_oracle_backward.restype = None
        lib.msda_oracle_decode_e4m3.argtypes = [vp, i64, vp]
        lib.msda_oracle_encode_e4m3.argtypes = [vp, i64, vp]
        lib.msda_oracle_encode_e4m3_exhaustive.argtypes = [vp, i64, vp]
        lib.msda_oracle_num_threads.restype = i32
        _lib = lib
    return _lib


def _f64(x) -> np.ndarray:
    if hasattr(x, "detach"):
        x = x.detach().cpu().double().numpy()
    return np.ascontiguousarray(x, dtype=np.float64)


def _i32(x) -> np.ndarray:
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(x, dtype=np.int32)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims(feat, shapes, loc, w):
    B, R, C = feat.shape
    N, L = shapes.shape[0], shapes.shape[1]
    A, P = loc.shape[1], loc.shape[2]
    G = w.shape[-1]
    assert loc.shape == (B, A, P, N, 2), loc.shape
    assert w.shape == (B, A, P, N, L, G), w.shape
    assert C % G == 0
    return B, N, L, A, P, C, G, R


def num_threads() -> int:
    return int(_load().msda_oracle_num_threads())


def forward(feat, spatial_shapes, level_start_index, sampling_loc, weights,
            nthreads: int = 0) -> np.ndarray:
    """out[B, A, C] in float64. Inputs are widened exactly to double first."""
    lib = _load()
    feat, loc, w = _f64(feat), _f64(sampling_loc), _f64(weights)
    shapes, starts = _i32(spatial_shapes), _i32(level_start_index)
    B, N, L, A, P, C, G, R = _dims(feat, shapes, loc, w)
    out = np.empty((B, A, C), dtype=np.float64)
    lib.msda_oracle_forward(B, N, L, A, P, C, G, R, _ptr(feat), _ptr(shapes), _ptr(starts),
                            _ptr(loc), _ptr(w), _ptr(out), int(nthreads))
    return out


def backward(feat, spatial_shapes, level_start_index, sampling_loc, weights, grad_out,
             need_feat: bool = True, need_loc: bool = True, need_w: bool = True,
             nthreads: int = 0):
    """(grad_feat, grad_loc, grad_w) in float64; a gradient not asked for is None."""
    lib = _load()
    feat, loc, w, go = _f64(feat), _f64(sampling_loc), _f64(weights), _f64(grad_out)
    shapes, starts = _i32(spatial_shapes), _i32(level_start_index)
    B, N, L, A, P, C, G, R = _dims(feat, shapes, loc, w)
    assert go.shape == (B, A, C)
    gf = np.empty_like(feat) if need_feat else None
    gl = np.empty_like(loc) if need_loc else None
    gw = np.empty_like(w) if need_w else None
    lib.msda_oracle_backward(B, N, L, A, P, C, G, R, _ptr(feat), _ptr(shapes), _ptr(starts),
                             _ptr(loc), _ptr(w), _ptr(go), _ptr(gf), _ptr(gl), _ptr(gw),
                             int(nthreads))
    return gf, gl, gw


def decode_e4m3(codes) -> np.ndarray:
    """OCP E4M3 codes (uint8, any shape) to float64."""
    lib = _load()
    if hasattr(codes, "detach"):
        codes = codes.detach().cpu().view(__import__("torch").uint8).numpy()
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    out = np.empty(c.shape, dtype=np.float64)
    lib.msda_oracle_decode_e4m3(_ptr(c), c.size, _ptr(out))
    return out


def encode_e4m3(x) -> np.ndarray:
    """float32 values to OCP E4M3 codes: clamp to +-448, round to nearest even."""
    lib = _load()
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    v = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(v.shape, dtype=np.uint8)
    lib.msda_oracle_encode_e4m3(_ptr(v), v.size, _ptr(out))
    return out


def _level_rows(spatial_shapes, level_start_index):
    shapes, starts = _i32(spatial_shapes), _i32(level_start_index)
    N, L = shapes.shape[0], shapes.shape[1]
    rows = [[] for _ in range(L)]
    for n in range(N):
        for l in range(L):
            s0 = int(starts[n, l])
            rows[l].append((s0, s0 + int(shapes[n, l, 0]) * int(shapes[n, l, 1])))
    return rows


def quantize_fp8_per_level(feat, spatial_shapes, level_start_index):
    """Per-level symmetric FP8 quantisation of feat [B, R, C] (float32).

    scale_l = amax_l / 448 in float32, amax over every batch item, camera and
    channel of level l (1 if the level is all zero); code = RNE(clamp(x /
    scale_l, +-448)) with the quotient formed in float32. Rows in no region get
    code 0. Returns (codes uint8 [B, R, C], scales float32 [L]).
    """
    if hasattr(feat, "detach"):
        feat = feat.detach().cpu().float().numpy()
    x = np.ascontiguousarray(feat, dtype=np.float32)
    levels = _level_rows(spatial_shapes, level_start_index)
    codes = np.zeros(x.shape, dtype=np.uint8)
    scales = np.empty(len(levels), dtype=np.float32)
    for l, regions in enumerate(levels):
        amax = np.float32(0.0)
        for r0, r1 in regions:
            if r1 > r0:
                amax = max(amax, np.float32(np.abs(x[:, r0:r1, :]).max()))
        scale = np.float32(amax / np.float32(448.0)) if amax > 0 else np.float32(1.0)
        scales[l] = scale
        for r0, r1 in regions:
            q = (x[:, r0:r1, :] / scale).astype(np.float32)
            codes[:, r0:r1, :] = encode_e4m3(q)
    return codes, scales


def dequantize_fp8(codes, scales, spatial_shapes, level_start_index) -> np.ndarray:
    """code * scale_l in float64 (exact); rows in no region decode to 0."""
    vals = decode_e4m3(codes)
    out = np.zeros(vals.shape, dtype=np.float64)
    sc = np.asarray(scales, dtype=np.float32).astype(np.float64)
    for l, regions in enumerate(_level_rows(spatial_shapes, level_start_index)):
        for r0, r1 in regions:
            out[:, r0:r1, :] = vals[:, r0:r1, :] * sc[l]
    return out
