"""FP64 oracle of the keypoint projection step upstream of MSDA, and of the
visible-view (sparse) form of MSDA.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU-baseline leg may use it.

What is computed (paper Sec. 3.1 and Sec. 3.2):

* Each anchor carries a 3D box state (x, y, z, w, l, h, yaw, vx, vy, vz)
  (Sec. 3.1 lists these as the predicted quantities) and P keypoints given
  as offsets in the box frame, in units of the box size (fixed geometric and
  learned keypoints, Sec. 3.2). A keypoint's world position is the box
  centre plus the yaw rotation (about the vertical z axis) of the offset
  scaled by (w, l, h), shifted by the velocity times the time offset dt: the
  motion compensation of Sec. 3.2.
* Each world point is projected into camera n with its 3x4 projection
  matrix (intrinsics times extrinsics, Sec. 3.1): (u', v', d) = M_n [X 1].
  With d > DEPTH_EPS the pixel is (u'/d, v'/d) and the normalised sampling
  location divides it by the camera's image width and height; a point at or
  behind the camera gets the location BEHIND (outside every level, so MSDA
  skips it).
* An anchor is visible in camera n when at least one of its keypoints lands
  in front of the camera and inside the image (0 <= px < W_img, 0 <= py <
  H_img). The sparse form of MSDA sums only over visible (anchor, camera)
  pairs; the gradients of invisible pairs' locations and weights are zero.

Parity status: pinned by the CPU tests (closed-form cameras and rotations,
the motion shift, points behind the camera, the sparse form against the
dense oracle with the invisible pairs' weights set to zero).
"""
from __future__ import annotations

import numpy as np

from . import backward as _dense_backward
from . import forward as _dense_forward

DEPTH_EPS = 1e-5
BEHIND = -2.0


def keypoints_world(anchors, keypoints, dt: float) -> np.ndarray:
    """World positions [B, A, P, 3] of the keypoints of anchors [B, A, 10]
    (x, y, z, w, l, h, yaw, vx, vy, vz); keypoints [B, A, P, 3] box-frame
    offsets in units of (w, l, h)."""
    a = np.asarray(anchors, dtype=np.float64)
    k = np.asarray(keypoints, dtype=np.float64)
    B, A, P, _ = k.shape
    out = np.zeros((B, A, P, 3))
    for b in range(B):
        for i in range(A):
            x, y, z, w, l, h, yaw, vx, vy, vz = a[b, i]
            c, s = np.cos(yaw), np.sin(yaw)
            for p in range(P):
                ox, oy, oz = k[b, i, p, 0] * w, k[b, i, p, 1] * l, k[b, i, p, 2] * h
                out[b, i, p, 0] = x + (c * ox - s * oy) + dt * vx
                out[b, i, p, 1] = y + (s * ox + c * oy) + dt * vy
                out[b, i, p, 2] = z + oz + dt * vz
    return out


def project_points(points, projection, image_hw):
    """points [B, A, P, 3] through projection [B, N, 3, 4] -> (pixel [B, A, P,
    N, 2], depth [B, A, P, N]); image_hw [N, 2] is unused here (kept for a
    uniform signature)."""
    pts = np.asarray(points, dtype=np.float64)
    M = np.asarray(projection, dtype=np.float64)
    B, A, P, _ = pts.shape
    N = M.shape[1]
    pix = np.zeros((B, A, P, N, 2))
    depth = np.zeros((B, A, P, N))
    for b in range(B):
        for n in range(N):
            for i in range(A):
                for p in range(P):
                    X = np.append(pts[b, i, p], 1.0)
                    h = M[b, n] @ X
                    depth[b, i, p, n] = h[2]
                    if h[2] > DEPTH_EPS:
                        pix[b, i, p, n] = (h[0] / h[2], h[1] / h[2])
    return pix, depth


def project_keypoints(anchors, keypoints, dt, projection, image_hw):
    """(sampling_loc [B, A, P, N, 2] normalised, visible [B, A, N] bool)."""
    pts = keypoints_world(anchors, keypoints, dt)
    pix, depth = project_points(pts, projection, image_hw)
    hw = np.asarray(image_hw, dtype=np.float64)          # [N, 2] (H, W)
    front = depth > DEPTH_EPS
    loc = np.full(pix.shape, BEHIND)
    W = hw[:, 1][None, None, None, :]
    H = hw[:, 0][None, None, None, :]
    loc[..., 0] = np.where(front, pix[..., 0] / W, BEHIND)
    loc[..., 1] = np.where(front, pix[..., 1] / H, BEHIND)
    inside = front & (pix[..., 0] >= 0) & (pix[..., 0] < W) & (pix[..., 1] >= 0) & \
        (pix[..., 1] < H)
    visible = inside.any(axis=2)                            # over keypoints
    return loc, visible


def _masked_weights(weights, visible):
    w = np.asarray(weights.numpy() if hasattr(weights, "numpy") else weights,
                   dtype=np.float64).copy()
    vis = np.asarray(visible, dtype=bool)                   # [B, A, N]
    w *= vis[:, :, None, :, None, None]
    return w


def forward_visible(feat, spatial_shapes, level_start_index, sampling_loc, weights, visible):
    """Sparse MSDA: the dense sum restricted to the visible (anchor, camera)
    pairs, i.e. the dense operator with those pairs' weights set to zero."""
    return _dense_forward(feat, spatial_shapes, level_start_index, sampling_loc,
                          _masked_weights(weights, visible))


def backward_visible(feat, spatial_shapes, level_start_index, sampling_loc, weights, visible,
                     grad_out):
    """Gradients of the sparse form: grad_feat of the masked dense operator;
    grad_loc and grad_w of visible pairs from it, zero for invisible pairs
    (they take no part in the sparse sum)."""
    gf, gl, gw = _dense_backward(feat, spatial_shapes, level_start_index, sampling_loc,
                                 _masked_weights(weights, visible), grad_out)
    vis = np.asarray(visible, dtype=bool)
    gl = gl * vis[:, :, None, :, None]
    gw = gw * vis[:, :, None, :, None, None]
    return gf, gl, gw


def _scores(view_score, visible):
    s = np.asarray(view_score.numpy() if hasattr(view_score, "numpy") else view_score,
                   dtype=np.float64)
    return s * np.asarray(visible, dtype=bool)


def forward_fused(feat, spatial_shapes, level_start_index, sampling_loc, weights, visible,
                  view_score):
    """Visibility-weighted fusion (Sec. 3.2, Eq. 2): f = sum_n v_n g_n / sum_n
    v_n over the visible cameras, g_n the anchor's aggregated feature in
    camera n alone (the visible-view sum restricted to camera n); f = 0 when
    the scores of the visible cameras sum to 0. Also returns the per-camera
    features g [B, A, N, C]."""
    vis = np.asarray(visible, dtype=bool)
    B, A, N = vis.shape
    g = []
    for n in range(N):
        only = np.zeros_like(vis)
        only[:, :, n] = vis[:, :, n]
        g.append(forward_visible(feat, spatial_shapes, level_start_index, sampling_loc, weights,
                                 only))
    g = np.stack(g, axis=2)                                  # [B, A, N, C]
    v = _scores(view_score, vis)
    V = v.sum(axis=2)                                       # [B, A]
    safe = np.where(V > 0, V, 1.0)
    f = (v[..., None] * g).sum(axis=2) / safe[..., None]
    f[V <= 0] = 0.0
    return f, g


def backward_fused(feat, spatial_shapes, level_start_index, sampling_loc, weights, visible,
                   view_score, grad_out):
    """Gradients of forward_fused: the visible-view gradients with grad_out
    scaled per camera by v_n / V (grad_feat, grad_loc, grad_weights), and
    grad_score[b, a, n] = <grad_out, g_n - f> / V for visible cameras (0
    otherwise, and 0 when V = 0)."""
    vis = np.asarray(visible, dtype=bool)
    v = _scores(view_score, vis)
    V = v.sum(axis=2)
    vt = np.where(V[..., None] > 0, v / np.where(V > 0, V, 1.0)[..., None], 0.0)   # [B, A, N]
    # the fused output is the visible-view operator with weights w * vt
    w = np.asarray(weights.numpy() if hasattr(weights, "numpy") else weights, dtype=np.float64)
    w_eff = w * vt[:, :, None, :, None, None]
    gf, gl, gw_eff = backward_visible(feat, spatial_shapes, level_start_index, sampling_loc,
                                      w_eff, vis, grad_out)
    # d f / d w = vt * (d out_visible / d w_eff): grad_w = vt * raw grad_w
    _, _, gw_raw = backward_visible(feat, spatial_shapes, level_start_index, sampling_loc, w,
                                    vis, grad_out)
    gw = gw_raw * vt[:, :, None, :, None, None]
    f, g = forward_fused(feat, spatial_shapes, level_start_index, sampling_loc, weights, vis,
                         view_score)
    go = np.asarray(grad_out, dtype=np.float64)
    dots = np.einsum("bac,banc->ban", go, g) - np.einsum("bac,bac->ba", go, f)[..., None]
    gs = np.where(vis & (V[..., None] > 0), dots / np.where(V > 0, V, 1.0)[..., None], 0.0)
    return gf, gl, gw, gs
