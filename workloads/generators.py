"""Seeded scene and camera generators for the five benchmark workloads.

Every array is drawn in float64 from ``np.random.default_rng(1000 * cfg + purpose)``
(PCG64) and cast to float32 once, so the oracle and the HIP path receive the
same bits.  Purposes: 0 = scene, 1 = target image, 2 = finite-difference subset,
3 = sampled parity pixels.

Layouts (structure of arrays, float32, C-contiguous):
  mean          [3][N]      world position x, y, z
  log_scale     [3][N]      per-axis log standard deviation
  quat          [4][N]      rotation quaternion (w, x, y, z), not normalised
  opacity_logit [N]
  sh            [K][3][N]   K = (degree + 1)^2 colour coefficients per channel

Cameras are pinhole, world -> camera ``x_c = R x_w + t`` with OpenCV axes
(x right, y down, z forward) and R stored row-major.

The five recipes follow the workloads named for the rasterizer benchmark: a
tiny single view, a single full-HD view, a 6-camera ring rig in a street
corridor, an uneven-resolution keyframe window and a large street scene.  The
paper's own datasets are not available; these synthetic street corridors stand
in for its road scenes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np


@dataclasses.dataclass
class Camera:
    R: np.ndarray  # (3, 3) float32, row-major, world -> camera
    t: np.ndarray  # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_row(self) -> np.ndarray:
        """18 float32 words: R[9], t[3], fx, fy, cx, cy, then width and height
        stored as int32 bit patterns (the C struct layout)."""
        row = np.zeros(18, dtype=np.float32)
        row[0:9] = self.R.reshape(-1)
        row[9:12] = self.t
        row[12:16] = (self.fx, self.fy, self.cx, self.cy)
        row[16:18] = np.array([self.width, self.height], dtype=np.int32).view(np.float32)
        return row


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def arrays(self):
        return dict(mean=self.mean, log_scale=self.log_scale, quat=self.quat,
                    opacity_logit=self.opacity_logit, sh=self.sh)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.mean[:, idx]),
                     np.ascontiguousarray(self.log_scale[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]),
                     np.ascontiguousarray(self.opacity_logit[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]),
                     self.sh_degree)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def _camera(cam_to_world: np.ndarray, centre: np.ndarray, f: float, w: int, h: int) -> Camera:
    """Pose from a camera->world rotation and a centre (world coordinates)."""
    r = cam_to_world.T
    t = -r @ centre
    return Camera(_f32(r), _f32(t), float(np.float32(f)), float(np.float32(f)),
                  float(np.float32(w / 2.0)), float(np.float32(h / 2.0)), int(w), int(h))


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree, dc_colour=False):
    k = (degree + 1) ** 2
    sh = np.empty((k, 3, n), dtype=np.float64)
    if dc_colour:
        # The colour itself is drawn U[0,1]; its degree-0 coefficient is
        # (colour - 0.5) / Y_0 with Y_0 = 1 / (2 sqrt(pi)).
        sh[0] = (rng.uniform(0.0, 1.0, (3, n)) - 0.5) * (2.0 * math.sqrt(math.pi))
    else:
        sh[0] = rng.uniform(0.0, 1.0, (3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, 0.2, (k - 1, 3, n))
    return sh


def _corridor(rng, n, z0, z1, half_width, facade_height, height_decay=None, ground_frac=0.4):
    """Street corridor: a ground plane 1.6 m below the rig plus two facades."""
    n_ground = int(round(n * ground_frac))
    n_facade = n - n_ground
    mean = np.empty((3, n), dtype=np.float64)
    mean[0, :n_ground] = rng.uniform(-half_width, half_width, n_ground)
    mean[1, :n_ground] = 1.6 + rng.normal(0.0, 0.05, n_ground)
    mean[2, :n_ground] = rng.uniform(z0, z1, n_ground)
    side = np.where(rng.uniform(0.0, 1.0, n_facade) < 0.5, -1.0, 1.0)
    mean[0, n_ground:] = side * half_width + rng.normal(0.0, 0.05, n_facade)
    if height_decay is None:
        h = rng.uniform(0.0, facade_height, n_facade)
    else:
        # exponential density in height, truncated at the facade height
        u = rng.uniform(0.0, 1.0, n_facade)
        h = -height_decay * np.log1p(-u * (1.0 - math.exp(-facade_height / height_decay)))
    mean[1, n_ground:] = 1.6 - h
    mean[2, n_ground:] = rng.uniform(z0, z1, n_facade)
    perm = rng.permutation(n)
    return mean[:, perm]


def _ring(centre, n_cams, yaw_step_deg, radius, f, w, h, rng=None, jitter_deg=0.0, res_choices=None):
    cams = []
    for k in range(n_cams):
        yaw = math.radians(k * yaw_step_deg)
        rot = _rot_y(yaw)
        if rng is not None and jitter_deg > 0.0:
            j = np.radians(rng.uniform(-jitter_deg, jitter_deg, 3))
            rot = rot @ _rot_y(j[0]) @ _rot_x(j[1]) @ _rot_z(j[2])
        c = np.asarray(centre, dtype=np.float64) + radius * np.array([math.sin(yaw), 0.0, math.cos(yaw)])
        ww, hh, ff = w, h, f
        if res_choices is not None:
            ww, hh = res_choices[int(rng.integers(0, len(res_choices)))]
            ff = 0.75 * ww
        cams.append(_camera(rot, c, ff, ww, hh))
    return cams


def _scene(mean, rng, n, ls_mu, ls_sigma, op_sigma, degree, dc_colour=False):
    return Scene(
        mean=_f32(mean),
        log_scale=_f32(rng.normal(ls_mu, ls_sigma, (3, n))),
        quat=_f32(_random_quats(rng, n)),
        opacity_logit=_f32(rng.normal(0.0, op_sigma, n)),
        sh=_f32(_sh(rng, n, degree, dc_colour)),
        sh_degree=degree,
    )


def _cfg1(rng, scale=1.0):
    n = max(1, int(round(2000 * scale)))
    mean = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    scene = Scene(
        mean=_f32(mean),
        log_scale=_f32(rng.normal(-3.0, 0.3, (3, n))),
        quat=_f32(_random_quats(rng, n)),
        opacity_logit=_f32(rng.normal(0.0, 1.0, n)),
        sh=_f32(_sh(rng, n, 0, dc_colour=True)),
        sh_degree=0,
    )
    cams = [_camera(np.eye(3), np.zeros(3), 60.0, 64, 48)]
    return scene, cams


def _cfg2(rng, scale=1.0):
    n = max(1, int(round(500_000 * scale)))
    mean = np.stack([rng.uniform(-20, 20, n), rng.uniform(-5, 5, n), rng.uniform(1, 41, n)])
    scene = _scene(mean, rng, n, -4.0, 0.5, 1.5, 3)
    cams = [_camera(np.eye(3), np.zeros(3), 1400.0, 1920, 1080)]
    return scene, cams


def _cfg3(rng, scale=1.0):
    n = max(1, int(round(1_000_000 * scale)))
    mean = _corridor(rng, n, -50.0, 50.0, 10.0, 12.0)
    scene = _scene(mean, rng, n, -3.5, 0.6, 1.5, 3)
    cams = _ring(np.zeros(3), 6, 60.0, 0.1, 1200.0, 1600, 900)
    return scene, cams


def _cfg4(rng, scale=1.0):
    n = max(1, int(round(2_000_000 * scale)))
    mean = _corridor(rng, n, -30.0, 30.0, 10.0, 12.0)
    scene = _scene(mean, rng, n, -3.5, 0.6, 1.5, 3)
    cams = []
    res = [(960, 540), (1280, 720), (1920, 1080)]
    for fr, zc in enumerate(np.linspace(-15.0, 15.0, 8)):
        cams += _ring(np.array([0.0, 0.0, zc]), 5, 72.0, 0.1, None, None, None,
                      rng=rng, jitter_deg=5.0, res_choices=res)
    return scene, cams


def _cfg5(rng, scale=1.0):
    n = max(1, int(round(6_000_000 * scale)))
    mean = _corridor(rng, n, -200.0, 200.0, 15.0, 30.0, height_decay=5.0)
    scene = _scene(mean, rng, n, -3.5, 0.6, 1.5, 3)
    cams = []
    for fr in range(4):
        cams += _ring(np.array([0.0, 0.0, 2.0 * fr]), 6, 60.0, 0.1, 1440.0, 1920, 1080)
    return scene, cams


CONFIGS = {
    1: ("single_view_64x48_2k", _cfg1),
    2: ("single_view_1920x1080_500k", _cfg2),
    3: ("rig6_1600x900_1M", _cfg3),
    4: ("window40_mixed_res_2M", _cfg4),
    5: ("street24_1920x1080_6M", _cfg5),
}


def make_insert_inputs(sizes, seed, detail_kept=0.3):
    """Ground truth, render and z-depth per view for the insertion step:
    the ground truth is a smooth field (a few random sinusoids) plus sharp
    detail (random axis-aligned rectangles and single-pixel dots of random
    colour); the render keeps the field and `detail_kept` of the detail; the
    depth is a smooth field between 3 and 30.  Planar [3][h][w] float32 per
    view, depth [h][w]."""
    rng = np.random.default_rng(seed)
    gts, rds, depths = [], [], []
    for w, h in sizes:
        y, x = np.mgrid[0:h, 0:w].astype(np.float64)
        base = np.zeros((3, h, w))
        for _ in range(4):
            fx, fy = rng.uniform(0.5, 4.0, 2) * 2 * np.pi / np.array([w, h])
            ph = rng.uniform(0, 2 * np.pi)
            base += rng.uniform(0.02, 0.1, (3, 1, 1)) * np.sin(fx * x + fy * y + ph)[None]
        base += 0.5
        detail = np.zeros((3, h, w))
        for _ in range(max(1, w * h // 4000)):
            x0, y0 = int(rng.integers(0, w)), int(rng.integers(0, h))
            x1, y1 = min(w, x0 + int(rng.integers(2, 40))), min(h, y0 + int(rng.integers(2, 40)))
            detail[:, y0:y1, x0:x1] = rng.uniform(-0.8, 0.8, (3, 1, 1))
        n_dots = max(1, w * h // 200)
        detail[:, rng.integers(0, h, n_dots), rng.integers(0, w, n_dots)] += rng.uniform(-1.5, 1.5, (3, n_dots))
        gts.append(_f32(base + detail))
        rds.append(_f32(base + detail_kept * detail))
        dz = 16.5 + 13.5 * np.sin(2 * np.pi * x / max(w, 2) * rng.uniform(0.2, 1.0)) * np.cos(
            2 * np.pi * y / max(h, 2) * rng.uniform(0.2, 1.0))
        depths.append(_f32(dz))
    return gts, rds, depths


# Rig layout of each workload's views, frame-major: (frames, cameras per frame).
RIG_LAYOUT = {1: (1, 1), 2: (1, 1), 3: (1, 6), 4: (8, 5), 5: (4, 6)}


def config_names():
    return {k: v[0] for k, v in CONFIGS.items()}


def make_config(cfg: int, scale: float = 1.0):
    """Scene and camera list of workload ``cfg`` (1..5).  ``scale`` shrinks the
    Gaussian count for quick tests while keeping the cameras and the spatial
    distribution of the scene."""
    rng = np.random.default_rng(1000 * cfg + 0)
    return CONFIGS[cfg][1](rng, scale)


def make_target(cfg: int, cams: List[Camera]):
    """Uniform [0,1] target image per view, planar [3][H][W] float32."""
    rng = np.random.default_rng(1000 * cfg + 1)
    return [_f32(rng.uniform(0.0, 1.0, (3, c.height, c.width))) for c in cams]
