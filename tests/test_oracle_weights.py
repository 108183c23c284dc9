"""Pins of the weight-generation oracle (per-group softmax of logits over the
(keypoint, camera, level) entries, and MSDA composed with it) against closed
forms, torch's softmax, finite differences and the softmax's invariants."""
import math

import numpy as np
import torch

from oracle import weights as ow
from paper_2601_10819_amd import synth


def logits_like(p, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(p.weights.shape, generator=g, dtype=torch.float64) * scale


def test_closed_forms():
    # two entries per group with logits 0 and ln 3: weights 1/4 and 3/4
    x = np.zeros((1, 1, 2, 1, 1, 2))
    x[0, 0, 1, 0, 0, :] = math.log(3.0)
    w = ow.softmax_weights(x)
    np.testing.assert_allclose(w[0, 0, :, 0, 0, 0], [0.25, 0.75], rtol=1e-15)
    # equal logits: every weight is 1 / (P * Ncam * L)
    x = np.full((2, 3, 5, 4, 3, 8), 0.7)
    np.testing.assert_allclose(ow.softmax_weights(x), 1.0 / 60.0, rtol=1e-14)


def test_matches_torch_softmax_and_shift_invariance():
    p = synth.small(seed=3, B=2, cams=3, A=5, P=4)
    x = logits_like(p, 1, scale=3.0)
    w = ow.softmax_weights(x)
    B, A, P, N, L, G = x.shape
    ref = torch.softmax(x.reshape(B, A, P * N * L, G), dim=2).reshape(x.shape).numpy()
    np.testing.assert_allclose(w, ref, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(w.sum(axis=(2, 3, 4)), 1.0, rtol=1e-13)
    # adding a constant per (b, a, g) changes nothing
    c = torch.randn(B, A, 1, 1, 1, G, dtype=torch.float64) * 50
    np.testing.assert_allclose(ow.softmax_weights(x + c), w, rtol=1e-12, atol=1e-16)


def test_masked_entries():
    p = synth.small(seed=4, B=1, cams=2, A=3, P=3)
    x = logits_like(p, 2)
    mask = torch.rand(x.shape, generator=torch.Generator().manual_seed(5)) < 0.3
    mask[..., 0, 0, 0, :] = False                     # keep one entry per group
    xm = x.masked_fill(mask, -math.inf)
    w = ow.softmax_weights(xm)
    assert np.all(w[mask.numpy()] == 0.0)
    B, A, P, N, L, G = x.shape
    keep = ~mask.numpy()
    for b in range(B):
        for a in range(A):
            for g in range(G):
                sel = keep[b, a, ..., g]
                ref = torch.softmax(x[b, a, ..., g][torch.from_numpy(sel)], dim=0).numpy()
                np.testing.assert_allclose(w[b, a, ..., g][sel], ref, rtol=1e-13)


def test_logit_gradient_by_finite_differences(oracle_mod):
    p = synth.small(seed=6, B=1, cams=3, levels=((6, 7), (3, 4)), C=16, G=2, A=3, P=2)
    x = logits_like(p, 7).numpy()
    go = synth.grad_out_like(p, seed=8).numpy().astype(np.float64)
    gf, gl, gx = ow.backward_logits(p.feat, p.spatial_shapes, p.level_start_index,
                                    p.sampling_loc, x, go)

    def loss(xx):
        out = ow.forward_logits(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc, xx)
        return float((out * go).sum())

    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(12):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        d = np.zeros_like(x)
        d[idx] = h
        fd = (loss(x + d) - loss(x - d)) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-8 * max(1.0, abs(fd)), (idx, fd, gx[idx])
    # the logits' gradient sums to zero over each group (softmax is shift-invariant)
    s = gx.sum(axis=(2, 3, 4))
    assert np.all(np.abs(s) <= 1e-12 * np.abs(gx).sum(axis=(2, 3, 4)).max())
    # feat and locations see the generated weights only
    w = ow.softmax_weights(x)
    rgf, rgl, _ = oracle_mod.backward(p.feat, p.spatial_shapes, p.level_start_index,
                                      p.sampling_loc, w, go)
    np.testing.assert_array_equal(gf, rgf)
    np.testing.assert_array_equal(gl, rgl)
