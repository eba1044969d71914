"""Seeded synthetic scenes shaped like the paper's workloads.

This module only draws random inputs: Gaussian parameters, pinhole cameras,
per-view medium coefficients and L1 targets.  It holds none of the renderer's
arithmetic, so both the CPU oracle tests and the HIP path consume the same
arrays from here.

The paper measures on real underwater captures (SeaThru-NeRF scenes and its
own TableDB, Sec. "Datasets and Camera Pose Extraction"); those are not
available, so these scenes stand in for them with the sizes, value
distributions and view resolutions of the benchmark configurations:

* config 0: 1,000 Gaussians, x,y in [-1,1], z in [2,6], SH degree 0 with
  RGB ~ U(0,1), one 128x128 camera at the origin looking +z, f = 128.
* config 1: 300k Gaussians in the box scaled x2.25 (x,y in [-2.25,2.25],
  z in [1,10]), SH degree 3 with coefficients ~ N(0, 0.1), one 1600x1067 view
  with a random pose looking into the box, 60 degree horizontal field of view.
* config 2: as config 1 with 1M Gaussians and one 1920x1080 view.
* config 3: 1M Gaussians, 24 views of sizes drawn from {640x480, 1280x720,
  1920x1080, 1600x1067} on a seeded orbit of radius 8 around (0, 0, 5.5).
* config 4: 3M Gaussians, four 1920x1080 views on the same orbit.

Common draws: log-scales ~ N(-3, 0.5) per axis (scales are the log-normal
variate, rounded to FP32); quaternions are normalised N(0, I4) draws (uniform
rotations; the raw draw is what is stored); opacities are the logit-normal
variate sigmoid(N(0,1)); medium per view: B_d ~ U(0.05,0.5)^3,
B_b ~ U(0.05,0.5)^3, B_inf ~ U(0,0.3)^3.  The draw order is fixed: means,
log-scales, quaternions, opacity logits, SH, medium, cameras, target.

Arrays are structure-of-arrays FP32 planes: means[3][N], scales[3][N],
quats[4][N] (w, x, y, z), opacity[N], sh[(deg+1)^2 * 3][N] with plane index
coef * 3 + channel.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

VIEW_SIZES = ((640, 480), (1280, 720), (1920, 1080), (1600, 1067))
NEAR_Z = 0.2


@dataclasses.dataclass
class Camera:
    """Pinhole camera, world-to-camera x_c = R x_w + t; looks down +z, image y down."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float32
    t: np.ndarray  # (3,) float32
    near: float = NEAR_Z

    def as_tuple(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                tuple(float(v) for v in np.asarray(self.R, np.float32).reshape(9)),
                tuple(float(v) for v in np.asarray(self.t, np.float32).reshape(3)),
                self.near)


@dataclasses.dataclass
class Scene:
    means: np.ndarray       # (3, N) f32
    log_scales: np.ndarray  # (3, N) f32
    scales: np.ndarray      # (3, N) f32, the log-normal variate
    quats: np.ndarray       # (4, N) f32, raw (unnormalised) draw
    logits: np.ndarray      # (N,) f32
    opacity: np.ndarray     # (N,) f32, the logit-normal variate
    sh: np.ndarray          # ((deg+1)^2 * 3, N) f32
    sh_degree: int
    cameras: List[Camera]
    medium: np.ndarray      # (V, 9) f32: B_d[3], B_b[3], B_inf[3]
    targets: Optional[List[np.ndarray]] = None  # per view (3, H, W) f32

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_views(self) -> int:
        return len(self.cameras)


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def look_at(center, target, width, height, fov_scale=0.866, near=NEAR_Z) -> Camera:
    """Camera at `center` looking at `target`, world 'up' = -y, f = fov_scale * width."""
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    up = np.array([0.0, -1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    R = np.stack([r, dn, f])
    t = -R @ c
    fx = fov_scale * width
    return Camera(int(width), int(height), float(np.float32(fx)), float(np.float32(fx)),
                  float(np.float32(width / 2.0)), float(np.float32(height / 2.0)),
                  _f32(R), _f32(t), near)


def _gaussians(rng, n, lo, hi, sh_degree, sh_mode):
    means = rng.uniform(lo, hi, size=(n, 3)).T
    log_scales = rng.normal(-3.0, 0.5, size=(3, n))
    quats = rng.normal(0.0, 1.0, size=(4, n))
    logits = rng.normal(0.0, 1.0, size=n)
    ncoef = (sh_degree + 1) ** 2
    if sh_mode == "rgb":
        # Degree-0 colour drawn uniformly in [0,1]; stored as the DC coefficient
        # of a colour map c = 1/2 + Y00 * k with Y00 = 1/(2 sqrt(pi)).
        rgb = rng.uniform(0.0, 1.0, size=(3, n))
        sh = (rgb - 0.5) * (2.0 * math.sqrt(math.pi))
        if ncoef > 1:
            sh = np.concatenate([sh, np.zeros((3 * (ncoef - 1), n))], axis=0)
    else:
        sh = rng.normal(0.0, 0.1, size=(ncoef * 3, n))
    return dict(
        means=_f32(means), log_scales=_f32(log_scales), scales=_f32(np.exp(log_scales)),
        quats=_f32(quats), logits=_f32(logits), opacity=_f32(1.0 / (1.0 + np.exp(-logits))),
        sh=_f32(sh), sh_degree=sh_degree)


def _medium(rng, v):
    bd = rng.uniform(0.05, 0.5, size=(v, 3))
    bb = rng.uniform(0.05, 0.5, size=(v, 3))
    binf = rng.uniform(0.0, 0.3, size=(v, 3))
    return _f32(np.concatenate([bd, bb, binf], axis=1))


def _targets(rng, cams):
    return [_f32(rng.uniform(0.0, 1.0, size=(3, c.height, c.width))) for c in cams]


def _orbit(rng, nviews, sizes):
    cams = []
    for k in range(nviews):
        ang = 2.0 * math.pi * k / nviews + rng.uniform(-0.1, 0.1)
        h = rng.uniform(-1.0, 1.0)
        center = (8.0 * math.cos(ang), h, 5.5 + 8.0 * math.sin(ang))
        w, hh = sizes[k]
        cams.append(look_at(center, (0.0, 0.0, 5.5), w, hh))
    return cams


def _random_pose(rng, width, height):
    center = (rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.0))
    target = (rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 5.5)
    return look_at(center, target, width, height)


def make_scene(config: int, n: Optional[int] = None, width: Optional[int] = None,
               height: Optional[int] = None, n_views: Optional[int] = None,
               seed: Optional[int] = None, with_target: bool = True,
               view_sizes: Optional[Sequence] = None) -> Scene:
    """Build benchmark configuration `config` (0..4) with seed 1000 + config.

    `n`, `width`/`height`, `n_views` override the sizes (for parity tests that
    keep the distributions but must finish on the CPU oracle in seconds).
    """
    seed = 1000 + config if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    if config == 0:
        n = 1000 if n is None else n
        g = _gaussians(rng, n, (-1.0, -1.0, 2.0), (1.0, 1.0, 6.0), 0, "rgb")
        med = _medium(rng, 1)
        w = 128 if width is None else width
        h = 128 if height is None else height
        cams = [Camera(w, h, 128.0, 128.0, w / 2.0, h / 2.0,
                       np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    elif config in (1, 2):
        n = (300_000 if config == 1 else 1_000_000) if n is None else n
        g = _gaussians(rng, n, (-2.25, -2.25, 1.0), (2.25, 2.25, 10.0), 3, "normal")
        med = _medium(rng, 1)
        dw, dh = (1600, 1067) if config == 1 else (1920, 1080)
        cams = [_random_pose(rng, dw if width is None else width, dh if height is None else height)]
    elif config in (3, 4):
        n = (1_000_000 if config == 3 else 3_000_000) if n is None else n
        g = _gaussians(rng, n, (-2.25, -2.25, 1.0), (2.25, 2.25, 10.0), 3, "normal")
        v = (24 if config == 3 else 4) if n_views is None else n_views
        med = _medium(rng, v)
        if view_sizes is not None:
            sizes = [tuple(s) for s in view_sizes]
        elif config == 3:
            idx = rng.integers(0, len(VIEW_SIZES), size=v)
            sizes = [VIEW_SIZES[i] for i in idx]
        else:
            sizes = [(1920, 1080)] * v
        if width is not None:
            sizes = [(width, height)] * v
        cams = _orbit(rng, v, sizes)
    else:
        raise ValueError(f"unknown configuration {config}")
    tgt = _targets(rng, cams) if with_target else None
    return Scene(cameras=cams, medium=med, targets=tgt, **g)


def custom_scene(seed: int, n: int, sh_degree: int, width: int, height: int,
                 lo=(-1.0, -1.0, 2.0), hi=(1.0, 1.0, 6.0), f: Optional[float] = None,
                 log_scale_mean: float = -3.0, log_scale_std: float = 0.5,
                 sh_std: float = 0.1, pose: str = "origin") -> Scene:
    """Small scene with the benchmark distributions, for oracle and parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(lo, hi, size=(n, 3)).T
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(3, n))
    quats = rng.normal(0.0, 1.0, size=(4, n))
    logits = rng.normal(0.0, 1.0, size=n)
    ncoef = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, sh_std, size=(ncoef * 3, n))
    if sh_degree == 0:
        sh = (rng.uniform(0.0, 1.0, size=(3, n)) - 0.5) * (2.0 * math.sqrt(math.pi))
    med = _medium(rng, 1)
    f = float(width) if f is None else f
    if pose == "origin":
        cam = Camera(width, height, float(np.float32(f)), float(np.float32(f)),
                     width / 2.0, height / 2.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    else:
        cam = _random_pose(rng, width, height)
    g = dict(means=_f32(means), log_scales=_f32(log_scales), scales=_f32(np.exp(log_scales)),
             quats=_f32(quats), logits=_f32(logits), opacity=_f32(1.0 / (1.0 + np.exp(-logits))),
             sh=_f32(sh), sh_degree=sh_degree)
    tgt = _targets(rng, [cam])
    return Scene(cameras=[cam], medium=med, targets=tgt, **g)
