"""FP64 oracle of the weights' generation step: the per-group softmax that
turns weight logits into MSDA's weights, and MSDA composed with it.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU-baseline leg may use it.

What is computed (the attention-weight normalisation upstream of MSDA, Sec.
3.1 / Sec. 3.2; the benchmark workloads draw their weights this way):

* logits have MSDA's weight layout [B, A, P, Ncam, L, G]; for each (b, a, g)
  the weights over the P*Ncam*L (keypoint, camera, level) entries are
  w = exp(x - m) / sum exp(x - m), m the entries' maximum (the definition of
  the softmax; subtracting m changes nothing mathematically). A logit of
  -inf is a masked entry: weight 0.
* MSDA's gradient with respect to the logits is the softmax's Jacobian
  applied to the gradient with respect to the weights:
  d x = w * (d w - sum over the group of w * d w).

Parity status: pinned by the CPU tests (uniform logits, shift invariance,
torch's softmax, masked entries, finite differences of the composed
operator, and the zero group sums of the logits' gradient).
"""
from __future__ import annotations

import numpy as np

from . import backward as _msda_backward
from . import forward as _msda_forward

_GROUP_AXES = (2, 3, 4)          # (P, Ncam, L) of [B, A, P, Ncam, L, G]


def _f64(x) -> np.ndarray:
    if hasattr(x, "detach"):
        x = x.detach().cpu().double().numpy()
    return np.asarray(x, dtype=np.float64)


def softmax_weights(logits) -> np.ndarray:
    """w [B, A, P, Ncam, L, G] in float64 from the logits (same layout)."""
    x = _f64(logits)
    m = x.max(axis=_GROUP_AXES, keepdims=True)
    e = np.exp(x - m)
    return e / e.sum(axis=_GROUP_AXES, keepdims=True)


def softmax_grad(w, grad_w) -> np.ndarray:
    """Gradient with respect to the logits from the weights w and the
    gradient with respect to the weights."""
    w = _f64(w)
    gw = _f64(grad_w)
    return w * (gw - (w * gw).sum(axis=_GROUP_AXES, keepdims=True))


def forward_logits(feat, spatial_shapes, level_start_index, sampling_loc, logits) -> np.ndarray:
    """MSDA with the weights generated from the logits."""
    return _msda_forward(feat, spatial_shapes, level_start_index, sampling_loc,
                         softmax_weights(logits))


def backward_logits(feat, spatial_shapes, level_start_index, sampling_loc, logits, grad_out):
    """(grad_feat, grad_sampling_loc, grad_logits) of forward_logits."""
    w = softmax_weights(logits)
    gf, gl, gw = _msda_backward(feat, spatial_shapes, level_start_index, sampling_loc, w,
                                grad_out)
    return gf, gl, softmax_grad(w, gw)
