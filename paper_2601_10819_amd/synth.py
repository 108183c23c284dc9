"""Seeded synthetic inputs for multi-scale deformable aggregation (MSDA).

This module only draws random inputs of the right shapes and distributions.
It holds none of the operator's arithmetic, and both the HIP path and the
FP64 oracle consume what it produces.

The paper (Sec. 3.1, Sec. 3.2, Sec. 5.3) describes the operator's inputs:
per-camera multi-scale backbone feature maps and 3D anchor keypoints projected
into every camera. It does not state the shapes. The workloads below are
Sparse4D-like stand-ins for the paper's multi-camera scenes (its dataset and
trained weights are not available); every tensor is drawn from a seeded
``torch.Generator`` on the CPU.

Tensor layouts (all contiguous):
  feat               [B, R, C]            R rows per batch item, channels fastest
  spatial_shapes     [Ncam, L, 2] int32   (H, W) of level l of camera n
  level_start_index  [Ncam, L]    int32   first row of region (n, l) in a batch item
  sampling_loc       [B, A, P, Ncam, 2]   normalised (x, y) in [0, 1] = image
  weights            [B, A, P, Ncam, L, G]

Rows of a batch item are camera-major, then level, then row-major (y, x).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import torch

# Strides of the 4-level feature pyramid (FPN outputs at 1/4 ... 1/32).
PYRAMID_STRIDES = (4, 8, 16, 32)


def pyramid_levels(img_h: int, img_w: int, strides: Sequence[int] = PYRAMID_STRIDES):
    """(H, W) of each pyramid level for an input image of img_h x img_w."""
    return [(img_h // s, img_w // s) for s in strides]


@dataclasses.dataclass
class Problem:
    """One MSDA invocation's inputs, on the CPU, in FP32 / int32."""

    name: str
    feat: torch.Tensor
    spatial_shapes: torch.Tensor
    level_start_index: torch.Tensor
    sampling_loc: torch.Tensor
    weights: torch.Tensor

    @property
    def batch(self) -> int:
        return self.feat.shape[0]

    @property
    def rows(self) -> int:
        return self.feat.shape[1]

    @property
    def channels(self) -> int:
        return self.feat.shape[2]

    @property
    def num_cams(self) -> int:
        return self.spatial_shapes.shape[0]

    @property
    def num_levels(self) -> int:
        return self.spatial_shapes.shape[1]

    @property
    def num_anchors(self) -> int:
        return self.sampling_loc.shape[1]

    @property
    def num_points(self) -> int:
        return self.sampling_loc.shape[2]

    @property
    def groups(self) -> int:
        return self.weights.shape[-1]

    @property
    def samples(self) -> int:
        """Nominal sample count S = B*A*P*Ncam*L (out-of-range ones included)."""
        return self.batch * self.num_anchors * self.num_points * self.num_cams * self.num_levels

    def dims(self):
        return dict(B=self.batch, Ncam=self.num_cams, L=self.num_levels, A=self.num_anchors,
                    P=self.num_points, C=self.channels, G=self.groups, R=self.rows)


def layout(levels_per_cam: Sequence[Sequence[Tuple[int, int]]]):
    """Camera-major row layout: returns (spatial_shapes, level_start_index, R)."""
    ncam = len(levels_per_cam)
    nlev = len(levels_per_cam[0])
    shapes = torch.zeros(ncam, nlev, 2, dtype=torch.int32)
    starts = torch.zeros(ncam, nlev, dtype=torch.int32)
    r = 0
    for n, levs in enumerate(levels_per_cam):
        assert len(levs) == nlev
        for l, (h, w) in enumerate(levs):
            shapes[n, l, 0] = h
            shapes[n, l, 1] = w
            starts[n, l] = r
            r += h * w
    return shapes, starts, r


def _grouped_softmax_weights(gen, B, A, P, N, L, G):
    """Per-(b, a, g) softmax over the P*N*L N(0,1) logits (an upstream input)."""
    logits = torch.randn(B, A, P * N * L, G, generator=gen, dtype=torch.float32)
    w = torch.softmax(logits.double(), dim=2).float()
    return w.reshape(B, A, P, N, L, G).contiguous()


def _reject_near_grid(gen, loc, shapes, margin_px):
    """Redraw (u, v) of any (b, a, p, n) whose x = u*W - 0.5 or y = v*H - 0.5 lies
    within margin_px of an integer at any level of camera n (this includes the
    -1 and W edges). Keeps finite differences inside one bilinear cell."""
    B, A, P, N, _ = loc.shape
    sh = shapes.double()  # [N, L, 2]
    for _ in range(200):
        u = loc[..., 0].double().unsqueeze(-1)  # [B, A, P, N, 1]
        v = loc[..., 1].double().unsqueeze(-1)
        x = u * sh[:, :, 1] - 0.5
        y = v * sh[:, :, 0] - 0.5
        dx = (x - torch.round(x)).abs()
        dy = (y - torch.round(y)).abs()
        bad = ((dx < margin_px) | (dy < margin_px)).any(dim=-1)  # [B, A, P, N]
        nbad = int(bad.sum())
        if nbad == 0:
            return loc
        fresh = torch.rand(nbad, 2, generator=gen, dtype=torch.float32) * 1.1 - 0.05
        loc[bad] = fresh
    raise RuntimeError("grid-line rejection did not converge")


def _out_of_view_locs(gen, B, A, P, N, frac):
    """Each (b, a, p, n) is out of camera n's view with probability frac.
    Out-of-view points lie in a band beyond every level (u or v in
    [-1, -0.5] or [1.5, 2]); the rest are U[0, 1]^2."""
    loc = torch.rand(B, A, P, N, 2, generator=gen, dtype=torch.float32)
    out = torch.rand(B, A, P, N, generator=gen) < frac
    which = torch.randint(0, 2, (B, A, P, N), generator=gen)       # 0: u, 1: v
    side = torch.randint(0, 2, (B, A, P, N), generator=gen)        # 0: low, 1: high
    band = torch.rand(B, A, P, N, generator=gen, dtype=torch.float32) * 0.5
    val = torch.where(side == 0, -1.0 + band, 1.5 + band)
    for k in (0, 1):
        sel = out & (which == k)
        loc[..., k] = torch.where(sel, val, loc[..., k])
    return loc.contiguous()


def make_problem(name: str, B: int, cam_levels, C: int, G: int, A: int, P: int, seed: int,
                 loc_mode: str = "uniform", grid_margin_px: Optional[float] = None,
                 out_of_view: float = 0.25) -> Problem:
    """Draw one problem. cam_levels: per camera, the list of (H, W) per level."""
    gen = torch.Generator().manual_seed(seed)
    shapes, starts, R = layout(cam_levels)
    N, L = shapes.shape[0], shapes.shape[1]
    feat = torch.randn(B, R, C, generator=gen, dtype=torch.float32)
    if loc_mode == "uniform":
        loc = (torch.rand(B, A, P, N, 2, generator=gen, dtype=torch.float32) * 1.1 - 0.05).contiguous()
    elif loc_mode == "out_of_view":
        loc = _out_of_view_locs(gen, B, A, P, N, out_of_view)
    else:
        raise ValueError(loc_mode)
    if grid_margin_px is not None:
        loc = _reject_near_grid(gen, loc, shapes, grid_margin_px)
    w = _grouped_softmax_weights(gen, B, A, P, N, L, G)
    return Problem(name, feat, shapes, starts, loc, w)


# ---------------------------------------------------------------------------
# The five workloads. Sizes follow Sparse4D-style detectors: 13 keypoints per
# anchor, 256 channels in 8 groups, a 4-level stride-4..32 pyramid.
# ---------------------------------------------------------------------------

def tiny(seed: int = 0) -> Problem:
    """B=1, 2 cameras, 128x224 image, C=64, G=4, 128 anchors x 13 keypoints."""
    levs = pyramid_levels(128, 224)
    return make_problem("tiny_2cam_c64", 1, [levs] * 2, 64, 4, 128, 13, seed)


def sparse4d(seed: int = 0, anchors: int = 900) -> Problem:
    """B=1, 6 cameras, 256x704 image, C=256, G=8, 900 anchors x 13 keypoints;
    locations kept >= 1e-3 px from grid lines at every level."""
    levs = pyramid_levels(256, 704)
    return make_problem("sparse4d_6cam", 1, [levs] * 6, 256, 8, anchors, 13, seed,
                        grid_margin_px=1e-3)


def train16(seed: int = 0, anchors: int = 1800) -> Problem:
    """B=2, 16 cameras, 384x640 image, C=256, G=8, 1800 anchors x 13 keypoints,
    25% of keypoints out of each camera's view (features used in BF16)."""
    levs = pyramid_levels(384, 640)
    return make_problem("train_2x16cam", 2, [levs] * 16, 256, 8, anchors, 13, seed,
                        loc_mode="out_of_view", out_of_view=0.25)


def cam64(seed: int = 0, anchors: int = 900, cams: int = 64) -> Problem:
    """One scene of 64 cameras, 256x448 image, C=256, G=8, 900 anchors x 13
    keypoints (the 64-camera single-GPU workload)."""
    levs = pyramid_levels(256, 448)
    return make_problem("scene_64cam", 1, [levs] * cams, 256, 8, anchors, 13, seed)


BATCH_RESOLUTIONS = ((256, 448), (384, 640), (512, 896))


# ---------------------------------------------------------------------------
# Outside-in scene geometry: the inputs of the keypoint projection step.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SceneGeometry:
    """Inputs of the projection step (all FP32, CPU):
      anchors     [B, A, 10]   (x, y, z, w, l, h, yaw, vx, vy, vz), metres / rad / m/s
      keypoints   [B, A, P, 3] box-frame offsets in units of (w, l, h)
      dt          time offset of the motion compensation, seconds
      projection  [B, N, 3, 4] camera projection matrices (pixels)
      image_hw    [N, 2] int32 image height and width in pixels
    """

    anchors: torch.Tensor
    keypoints: torch.Tensor
    dt: float
    projection: torch.Tensor
    image_hw: torch.Tensor


# 7 fixed keypoints: the box centre and its 6 face centres
FIXED_KEYPOINTS = ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (-0.5, 0.0, 0.0), (0.0, 0.5, 0.0),
                   (0.0, -0.5, 0.0), (0.0, 0.0, 0.5), (0.0, 0.0, -0.5))


def _camera_matrix(eye, target, hfov, img_hw):
    """K [R | -R eye] of a pinhole camera at eye looking at target (z up in
    the world; camera x right, y down, z forward)."""
    eye = torch.as_tensor(eye, dtype=torch.float64)
    fwd = torch.as_tensor(target, dtype=torch.float64) - eye
    fwd = fwd / fwd.norm()
    right = torch.linalg.cross(fwd, torch.tensor([0.0, 0.0, 1.0], dtype=torch.float64))
    right = right / right.norm()
    down = torch.linalg.cross(fwd, right)
    R = torch.stack([right, down, fwd])
    H, W = img_hw
    f = (W / 2.0) / math.tan(hfov / 2.0)
    K = torch.tensor([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]], dtype=torch.float64)
    Rt = torch.cat([R, (-R @ eye)[:, None]], dim=1)
    return (K @ Rt).float()


def outside_in(seed: int = 0, B: int = 1, cams: int = 64, anchors: int = 900, P: int = 13,
               img_hw=(256, 448), area: float = 30.0, radius: float = 35.0,
               dt: float = 0.1) -> SceneGeometry:
    """An outside-in camera network: cams cameras on a ring of the given
    radius around a square area of half-width `area`, at heights U[5, 10] m,
    each aimed at a ground point uniform over the area with a horizontal
    field of view U[20, 40] degrees (at the defaults an anchor is seen by
    about 15 of 64 cameras); anchors uniform over the area (z U[0, 1.5])
    with sizes w U[0.5, 2], l U[0.5, 5], h U[1.5, 2.5], yaw U[0, 2 pi) and
    velocities N(0, 1.5) m/s (vertical x 0.1); the 7 fixed keypoints plus
    P - 7 learned offsets U[-0.5, 0.5]^3."""
    gen = torch.Generator().manual_seed(seed)
    u = lambda *shape: torch.rand(*shape, generator=gen, dtype=torch.float64)
    proj = torch.zeros(B, cams, 3, 4)
    for b in range(B):
        for n in range(cams):
            ang = 2 * math.pi * (n + float(u(1))) / cams
            eye = (radius * math.cos(ang), radius * math.sin(ang), 5.0 + 5.0 * float(u(1)))
            target = ((2 * float(u(1)) - 1) * area, (2 * float(u(1)) - 1) * area, 0.0)
            hfov = math.radians(20.0 + 20.0 * float(u(1)))
            proj[b, n] = _camera_matrix(eye, target, hfov, img_hw)
    a = torch.zeros(B, anchors, 10, dtype=torch.float64)
    a[..., 0] = (2 * u(B, anchors) - 1) * area
    a[..., 1] = (2 * u(B, anchors) - 1) * area
    a[..., 2] = 1.5 * u(B, anchors)
    a[..., 3] = 0.5 + 1.5 * u(B, anchors)
    a[..., 4] = 0.5 + 4.5 * u(B, anchors)
    a[..., 5] = 1.5 + 1.0 * u(B, anchors)
    a[..., 6] = 2 * math.pi * u(B, anchors)
    a[..., 7:10] = torch.randn(B, anchors, 3, generator=gen, dtype=torch.float64) * 1.5
    a[..., 9] *= 0.1
    k = torch.zeros(B, anchors, P, 3, dtype=torch.float64)
    nfix = min(P, len(FIXED_KEYPOINTS))
    k[:, :, :nfix] = torch.tensor(FIXED_KEYPOINTS[:nfix], dtype=torch.float64)
    if P > nfix:
        k[:, :, nfix:] = u(B, anchors, P - nfix, 3) - 0.5
    hw = torch.tensor([list(img_hw)] * cams, dtype=torch.int32)
    return SceneGeometry(a.float(), k.float(), dt, proj, hw)


def batched_scene_shapes(seed: int = 0, scenes: int = 12):
    """Per-scene (cams, (img_h, img_w), anchors) for the uneven multi-scene batch:
    cameras U{4..64}, resolution from three sizes, anchors U{300..1800}."""
    gen = torch.Generator().manual_seed(seed)
    out = []
    for _ in range(scenes):
        n = int(torch.randint(4, 65, (1,), generator=gen))
        r = int(torch.randint(0, 3, (1,), generator=gen))
        a = int(torch.randint(300, 1801, (1,), generator=gen))
        out.append((n, BATCH_RESOLUTIONS[r], a))
    return out


def batched(seed: int = 0, scenes: int = 12, scale_anchors: float = 1.0,
            max_cams: Optional[int] = None) -> List[Problem]:
    """The uneven multi-scene batch: 12 scenes, each its own Problem (B=1).
    scale_anchors / max_cams shrink the draw for small test cases."""
    out = []
    for i, (n, (h, w), a) in enumerate(batched_scene_shapes(seed, scenes)):
        if max_cams is not None:
            n = min(n, max_cams)
        a = max(1, int(round(a * scale_anchors)))
        levs = pyramid_levels(h, w)
        out.append(make_problem(f"scene{i}_{n}cam_{h}x{w}", 1, [levs] * n, 256, 8, a, 13,
                                seed * 1000 + 17 + i))
    return out


def small(seed: int, B=1, cams=2, levels=((6, 10), (3, 5)), C=32, G=4, A=5, P=3,
          loc_mode="uniform") -> Problem:
    """Small odd-shaped problems for exhaustive tests (ragged everything)."""
    return make_problem(f"small_s{seed}", B, [list(levels)] * cams, C, G, A, P, seed,
                        loc_mode=loc_mode)


def grad_out_like(problem: Problem, seed: int = 1) -> torch.Tensor:
    """Seeded N(0,1) upstream gradient of shape [B, A, C]."""
    gen = torch.Generator().manual_seed(seed)
    return torch.randn(problem.batch, problem.num_anchors, problem.channels, generator=gen,
                       dtype=torch.float32)


WORKLOADS = {
    "tiny": tiny,
    "sparse4d": sparse4d,
    "train16": train16,
    "cam64": cam64,
}
