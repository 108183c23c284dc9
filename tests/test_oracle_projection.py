"""Pins of the projection oracle (keypoints -> sampling locations and
visibility, paper Sec. 3.1 / Sec. 3.2) and of the visible-view (sparse) form
of MSDA, against closed forms and independent constructions."""
import math

import numpy as np
import pytest

from oracle import projection as proj
from paper_2601_10819_amd import synth


def anchor(x=0.0, y=0.0, z=0.0, w=1.0, l=1.0, h=1.0, yaw=0.0, vx=0.0, vy=0.0, vz=0.0):
    return np.array([[[x, y, z, w, l, h, yaw, vx, vy, vz]]], dtype=np.float64)


def test_keypoint_world_positions():
    a = anchor(1, 2, 3, w=2, l=4, h=6)
    k = np.array([[[[0, 0, 0], [0.5, 0, 0], [0, 0.5, 0], [0, 0, -0.5]]]], dtype=np.float64)
    got = proj.keypoints_world(a, k, 0.0)[0, 0]
    np.testing.assert_allclose(got, [[1, 2, 3], [2, 2, 3], [1, 4, 3], [1, 2, 0]], atol=1e-12)
    # a quarter turn of yaw takes the box's x axis to the world's y axis
    a = anchor(1, 2, 3, w=2, l=4, h=6, yaw=math.pi / 2)
    got = proj.keypoints_world(a, k, 0.0)[0, 0]
    np.testing.assert_allclose(got, [[1, 2, 3], [1, 3, 3], [-1, 2, 3], [1, 2, 0]], atol=1e-12)
    # motion compensation: every keypoint moves by dt * velocity
    a = anchor(1, 2, 3, w=2, l=4, h=6, yaw=0.3, vx=1.0, vy=-2.0, vz=0.5)
    base = proj.keypoints_world(anchor(1, 2, 3, w=2, l=4, h=6, yaw=0.3), k, 0.0)
    got = proj.keypoints_world(a, k, 0.1)
    np.testing.assert_allclose(got - base, np.broadcast_to([0.1, -0.2, 0.05], got.shape),
                               atol=1e-12)


def test_identity_and_pinhole_cameras():
    pts = np.array([[[[0.3, -0.4, 2.0], [1.0, 2.0, 4.0]]]])
    M = np.zeros((1, 1, 3, 4))
    M[0, 0, :, :3] = np.eye(3)
    pix, depth = proj.project_points(pts, M, [[1, 1]])
    np.testing.assert_allclose(pix[0, 0, :, 0], [[0.15, -0.2], [0.25, 0.5]], atol=1e-15)
    np.testing.assert_allclose(depth[0, 0, :, 0], [2.0, 4.0])
    # K [I | t]: f X / (Z + tz) + cx
    f, cx, cy, tz = 100.0, 50.0, 40.0, 5.0
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1]])
    M[0, 0] = K @ np.hstack([np.eye(3), [[0], [0], [tz]]])
    pix, _ = proj.project_points(pts, M, [[80, 100]])
    want = [[f * 0.3 / 7 + cx, f * -0.4 / 7 + cy], [f * 1 / 9 + cx, f * 2 / 9 + cy]]
    np.testing.assert_allclose(pix[0, 0, :, 0], want, atol=1e-12)


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World-to-camera [R | t] of a camera at eye looking at target (camera z
    forward, x right, y down), built here independently of the generator."""
    eye, target, up = map(lambda v: np.asarray(v, dtype=np.float64), (eye, target, up))
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return np.hstack([R, (-R @ eye)[:, None]]), x, y, z


def test_look_at_camera_principal_point_and_offsets():
    Rt, x, y, z = look_at([10.0, -4.0, 6.0], [0.0, 1.0, 0.5])
    f, cx, cy = 300.0, 224.0, 128.0
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1]])
    M = (K @ Rt)[None, None]
    eye = np.array([10.0, -4.0, 6.0])
    d = 7.0
    pts = np.stack([eye + d * z, eye + d * z + 0.5 * x, eye + d * z - 0.25 * y])[None, None]
    pix, depth = proj.project_points(pts, M, [[256, 448]])
    np.testing.assert_allclose(pix[0, 0, 0, 0], [cx, cy], atol=1e-9)
    np.testing.assert_allclose(pix[0, 0, 1, 0], [cx + f * 0.5 / d, cy], atol=1e-9)
    np.testing.assert_allclose(pix[0, 0, 2, 0], [cx, cy - f * 0.25 / d], atol=1e-9)
    np.testing.assert_allclose(depth[0, 0, :, 0], [d, d, d], atol=1e-9)


def test_behind_camera_and_visibility():
    Rt, x, y, z = look_at([0.0, 0.0, 0.0], [0.0, 10.0, 0.0])
    f = 100.0
    K = np.array([[f, 0, 50.0], [0, f, 40.0], [0, 0, 1]])
    M = (K @ Rt)[None, None]
    hw = [[80, 100]]
    # anchor 0 straight ahead (visible), 1 behind the camera, 2 in front but
    # outside the image, 3 with one keypoint inside and one outside
    anchors = np.array([[[0, 5, 0, 1, 1, 1, 0, 0, 0, 0],
                         [0, -5, 0, 1, 1, 1, 0, 0, 0, 0],
                         [40, 5, 0, 1, 1, 1, 0, 0, 0, 0],
                         [2.4, 5, 0, 2, 1, 1, 0, 0, 0, 0]]], dtype=np.float64)
    k = np.zeros((1, 4, 2, 3))
    k[0, :, 1, 0] = 0.5                                  # second keypoint: +0.5 w along x
    loc, vis = proj.project_keypoints(anchors, k, 0.0, M, hw)
    assert vis[0, :, 0].tolist() == [True, False, False, True]
    assert np.all(loc[0, 1] == proj.BEHIND)
    np.testing.assert_allclose(loc[0, 0, 0, 0], [0.5, 0.5], atol=1e-12)
    # anchor 3: centre at px = 50 + 100 * 2.4 / 5 = 98 (inside), keypoint 1 at
    # px = 50 + 100 * 3.4 / 5 = 118 (outside the 100-pixel width)
    np.testing.assert_allclose(loc[0, 3, :, 0, 0], [0.98, 1.18], atol=1e-12)


def test_sparse_form_sums_single_camera_problems(oracle_mod):
    """The visible-view sum equals the sum, over visible cameras, of the
    dense oracle run on each camera alone (its own regions and rows)."""
    p = synth.small(seed=21, B=2, cams=3, levels=((6, 7), (3, 4)), C=16, G=2, A=5, P=3)
    rng = np.random.default_rng(4)
    vis = rng.random((2, 5, 3)) < 0.6
    got = proj.forward_visible(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights, vis)
    want = np.zeros_like(got)
    feat = p.feat.numpy().astype(np.float64)
    for n in range(3):
        starts = p.level_start_index[n].numpy()
        shapes = p.spatial_shapes[n:n + 1].numpy()
        rows = [np.arange(s, s + h * w) for s, (h, w) in zip(starts, shapes[0])]
        sub = feat[:, np.concatenate(rows)]
        sub_starts = np.cumsum([0] + [h * w for h, w in shapes[0][:-1]])[None].astype(np.int32)
        single = oracle_mod.forward(sub, shapes, sub_starts,
                                    p.sampling_loc[:, :, :, n:n + 1].contiguous(),
                                    p.weights[:, :, :, n:n + 1].contiguous())
        want += single * vis[:, :, n][..., None]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    # all visible: the dense operator
    dense = oracle_mod.forward(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights)
    allv = proj.forward_visible(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                                p.weights, np.ones((2, 5, 3), dtype=bool))
    np.testing.assert_array_equal(allv, dense)


def test_sparse_backward_zero_for_invisible_pairs(oracle_mod):
    p = synth.small(seed=22, B=1, cams=4, C=8, G=2, A=6, P=2)
    vis = np.zeros((1, 6, 4), dtype=bool)
    vis[0, :, 1] = True
    vis[0, 2, 3] = True
    go = synth.grad_out_like(p, seed=3).numpy()
    gf, gl, gw = proj.backward_visible(p.feat, p.spatial_shapes, p.level_start_index,
                                       p.sampling_loc, p.weights, vis, go)
    assert np.all(gl[0][~vis[0][:, None, :].repeat(2, 1)] == 0)
    assert np.all(gw[:, :, :, 0] == 0) and np.all(gw[:, :, :, 2] == 0)
    assert np.any(gw[:, 2, :, 3] != 0) and np.all(gw[:, 3, :, 3] == 0)
    # Euler identity of the sparse form: <grad_w, w> = <grad_out, out>
    out = proj.forward_visible(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights, vis)
    e = float((out * go).sum())
    assert abs(float((gw * p.weights.numpy()).sum()) - e) <= 1e-12 * max(1.0, abs(e))
    assert abs(float((gf * p.feat.numpy()).sum()) - e) <= 1e-12 * max(1.0, abs(e))


def fused_case():
    p = synth.small(seed=23, B=2, cams=4, levels=((6, 7), (3, 4)), C=8, G=2, A=5, P=3)
    rng = np.random.default_rng(8)
    vis = rng.random((2, 5, 4)) < 0.7
    vis[0, 0] = False                                        # an anchor no camera sees
    score = rng.random((2, 5, 4))
    return p, vis, score


def test_fused_special_cases(oracle_mod):
    p, vis, score = fused_case()
    f, g = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, vis, score)
    assert np.all(f[0, 0] == 0)
    # equal scores: the mean of the visible cameras' features
    ones = np.ones_like(score)
    f1, _ = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights, vis, ones)
    sv = proj.forward_visible(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, vis)
    cnt = vis.sum(-1)
    np.testing.assert_allclose(f1[cnt > 0], (sv / np.maximum(cnt, 1)[..., None])[cnt > 0],
                               rtol=1e-12, atol=1e-13)
    # a one-hot score picks that camera's feature
    hot = np.zeros_like(score)
    hot[1, 2, 3] = 0.4
    vis2 = vis.copy()
    vis2[1, 2, 3] = True
    fh, gh = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                                p.weights, vis2, hot)
    np.testing.assert_allclose(fh[1, 2], gh[1, 2, 3], rtol=1e-14)
    # scaling every score of an anchor leaves the fusion unchanged
    f2, _ = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                               p.weights, vis, 3.5 * score)
    np.testing.assert_allclose(f2, f, rtol=1e-12, atol=1e-14)


def test_fused_gradients_by_finite_differences(oracle_mod):
    """grad_score and grad_w of the fusion against central differences of
    <grad_out, f> in FP64."""
    p, vis, score = fused_case()
    go = synth.grad_out_like(p, seed=6).numpy().astype(np.float64)
    gf, gl, gw, gs = proj.backward_fused(p.feat, p.spatial_shapes, p.level_start_index,
                                         p.sampling_loc, p.weights, vis, score, go)

    def loss(sc=score, w=p.weights.numpy()):
        f, _ = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                                  w, vis, sc)
        return float((f * go).sum())

    h = 1e-6
    for (b, a, n) in [(1, 2, 1), (0, 3, 2), (1, 4, 0), (0, 1, 3)]:
        d = np.zeros_like(score)
        d[b, a, n] = h
        fd = (loss(score + d) - loss(score - d)) / (2 * h)
        assert abs(fd - gs[b, a, n]) <= 1e-7 * max(1.0, abs(fd)), (b, a, n, fd, gs[b, a, n])
        if not vis[b, a, n]:
            assert gs[b, a, n] == 0.0
    w0 = p.weights.numpy().astype(np.float64)
    for idx in [(1, 2, 0, 1, 0, 1), (0, 3, 2, 2, 1, 0)]:
        d = np.zeros_like(w0)
        d[idx] = h
        fd = (loss(w=w0 + d) - loss(w=w0 - d)) / (2 * h)
        assert abs(fd - gw[idx]) <= 1e-7 * max(1.0, abs(fd)), (idx, fd, gw[idx])
    # the Euler identity in the features: f is linear in feat
    f, _ = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, p.sampling_loc,
                              p.weights, vis, score)
    e = float((f * go).sum())
    assert abs(float((gf * p.feat.numpy()).sum()) - e) <= 1e-12 * max(1.0, abs(e))


def test_fused_grad_loc_by_finite_differences(oracle_mod):
    """grad_sampling_loc of the fusion (Sec. 3.2, Eq. 2) against central
    differences of <grad_out, f> in FP64, at coordinates at least 1e-3 px
    from every grid line of the camera's levels (so the step stays inside one
    bilinear cell); coordinates of invisible pairs have an exactly zero
    gradient and no effect on f."""
    p, vis, score = fused_case()
    go = synth.grad_out_like(p, seed=7).numpy().astype(np.float64)
    _, gl, _, _ = proj.backward_fused(p.feat, p.spatial_shapes, p.level_start_index,
                                      p.sampling_loc, p.weights, vis, score, go)
    loc0 = p.sampling_loc.numpy().astype(np.float64)
    shapes = p.spatial_shapes.numpy()

    def loss(loc):
        f, _ = proj.forward_fused(p.feat, p.spatial_shapes, p.level_start_index, loc, p.weights,
                                  vis, score)
        return float((f * go).sum())

    def clear_of_grid(b, a, pp, n, k):
        # x = u*W - 0.5 (k = 0) or y = v*H - 0.5 (k = 1) at every level
        size = shapes[n, :, 1 - k].astype(np.float64)
        t = loc0[b, a, pp, n, k] * size - 0.5
        return bool(np.all(np.abs(t - np.round(t)) >= 1e-3))

    h = 1e-7
    rng = np.random.default_rng(9)
    checked_vis = checked_invis = 0
    B, A, P, N = loc0.shape[:4]
    for _ in range(400):
        idx = tuple(int(rng.integers(0, s)) for s in (B, A, P, N, 2))
        if not clear_of_grid(*idx):
            continue
        d = np.zeros_like(loc0)
        d[idx] = h
        fd = (loss(loc0 + d) - loss(loc0 - d)) / (2 * h)
        if vis[idx[:2] + (idx[3],)]:
            assert abs(fd - gl[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, gl[idx])
            checked_vis += 1
        else:
            assert gl[idx] == 0.0 and fd == 0.0, (idx, fd, gl[idx])
            checked_invis += 1
        if checked_vis >= 12 and checked_invis >= 3:
            break
    assert checked_vis >= 12 and checked_invis >= 3
    # a nonzero gradient somewhere, so the comparison above is not vacuous
    assert np.abs(gl).max() > 1e-3
