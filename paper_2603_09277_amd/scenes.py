"""Seeded synthetic scenes and cameras for the rasterizer and its oracle.

This module only draws inputs.  It holds none of the rasterizer's arithmetic:
no projection, binning, blending or entropy.  Both the HIP path and the FP64
oracle consume what it returns, so the two sides always see identical bits.

Workload recipe (the paper measures on Mip-NeRF 360 / Tanks & Temples / Deep
Blending, which are not available; these seeded scenes stand in for them with
the Gaussian counts the paper trains at, Sec. 5.3 and Tab. 1, 0.4M-3.3M):

* ``tiny``      2,000 Gaussians in front of one 128x128 pinhole camera, SH
                degree 0 with colours uniform in [0, 1].
* ``gmm``       a 64-cluster Gaussian-mixture point cloud in a 10-unit box,
                log-scales ~ N(-4, 0.7), SH degree 3 (DC ~ U[0, 1], higher
                bands ~ N(0, 0.05)), cameras on an orbit of radius 12.

Parameters are returned *activated*: scales are exp(log-scale), opacities are
sigmoid(logit).  Quaternions are (w, x, y, z) and are not normalised here.
Cameras use OpenCV axes (x right, y down, z forward); ``R``/``t`` map world to
camera coordinates, x_cam = R x_world + t.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Value of the l=0 real spherical harmonic, 1 / (2 sqrt(pi)).  Used only to
# express "colour uniform in [0, 1]" as a degree-0 coefficient (colour =
# Y00 * k + 0.5), which is how the tiny workload states its colours.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # (3, 3) float32, world -> camera, row-major
    t: np.ndarray            # (3,) float32
    near: float = 0.2

    def as_array(self) -> np.ndarray:
        """Flat float64 layout of the oracle (19 values).  Every value is first
        rounded to float32, the precision in which the GPU library receives a
        camera, so both sides see the same camera."""
        f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
        return np.concatenate([
            np.array([self.width, self.height], np.float64),
            f32([self.fx, self.fy, self.cx, self.cy]),
            f32(self.R).reshape(9),
            f32(self.t).reshape(3),
            f32([self.near]),
        ])


@dataclasses.dataclass
class Scene:
    means: np.ndarray        # (N, 3) float32
    scales: np.ndarray       # (N, 3) float32, > 0
    quats: np.ndarray        # (N, 4) float32, (w, x, y, z), unnormalised
    opacities: np.ndarray    # (N,)   float32 in (0, 1)
    sh: np.ndarray           # (N, K, 3) float32, K = (deg + 1)^2
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.scales[idx].copy(), self.quats[idx].copy(),
                     self.opacities[idx].copy(), self.sh[idx].copy(), self.sh_degree)

    def copy(self) -> "Scene":
        return self.subset(np.arange(self.n))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for OpenCV axes looking from ``eye`` at ``target``.

    ``up`` is the world direction that should appear up in the image, i.e.
    along the camera's -y axis.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    right = np.cross(f, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f], 0)
    t = -R @ eye
    return R.astype(np.float32), t.astype(np.float32)


def orbit_cameras(rng: np.random.Generator, resolutions, radius=12.0, focal_scale=0.8,
                  near=0.2) -> List[Camera]:
    """Cameras on a sphere around the origin, azimuth ~ U[0, 2pi), elevation
    ~ U[-15deg, 30deg], looking at the origin with world up +y."""
    cams = []
    for (w, h) in resolutions:
        az = rng.uniform(0.0, 2.0 * math.pi)
        el = math.radians(rng.uniform(-15.0, 30.0))
        eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
        R, t = look_at(eye)
        f = focal_scale * w
        cams.append(Camera(int(w), int(h), float(f), float(f), w / 2.0, h / 2.0, R, t, near))
    return cams


def random_quats(rng, n):
    return rng.standard_normal((n, 4)).astype(np.float32)


def tiny_scene(seed: int = 1, n: int = 2000):
    """2,000 Gaussians, one 128x128 camera (fx = fy = 128), SH degree 0."""
    rng = np.random.default_rng(seed)
    means = np.empty((n, 3), np.float32)
    means[:, 0:2] = rng.uniform(-1.0, 1.0, (n, 2))
    means[:, 2] = 4.0 + rng.uniform(-1.0, 1.0, n)
    scales = np.exp(rng.normal(-3.0, 0.5, (n, 3))).astype(np.float32)
    q = rng.standard_normal((n, 4))
    quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    opac = _sigmoid(rng.standard_normal(n)).astype(np.float32)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    sh = ((rgb - 0.5) / _Y00).astype(np.float32).reshape(n, 1, 3)
    cam = Camera(128, 128, 128.0, 128.0, 64.0, 64.0, np.eye(3, dtype=np.float32),
                 np.zeros(3, np.float32), 0.2)
    return Scene(means, scales, quats, opac, sh, 0), [cam]


def target_image(seed: int, height: int, width: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, (height, width, 3)).astype(np.float32)


def gmm_scene(seed: int, n: int, sh_degree: int = 3, n_clusters: int = 64, box: float = 10.0,
              cluster_sigma: float = 0.3, log_scale_mu: float = -4.0, log_scale_sigma: float = 0.7,
              opacity_logit_sigma: float = 1.5) -> Scene:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box / 2, box / 2, (n_clusters, 3))
    which = rng.integers(0, n_clusters, n)
    means = (centres[which] + cluster_sigma * rng.standard_normal((n, 3))).astype(np.float32)
    scales = np.exp(rng.normal(log_scale_mu, log_scale_sigma, (n, 3))).astype(np.float32)
    q = rng.standard_normal((n, 4))
    quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    opac = _sigmoid(rng.normal(0.0, opacity_logit_sigma, n)).astype(np.float32)
    K = (sh_degree + 1) ** 2
    sh = np.empty((n, K, 3), np.float32)
    sh[:, 0, :] = rng.uniform(0.0, 1.0, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, (n, K - 1, 3))
    return Scene(means, scales, quats, opac, sh, sh_degree)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 to the nearest bfloat16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out.reshape(x.shape)


# --------------------------------------------------------------------------- #
# Named workloads
# --------------------------------------------------------------------------- #

def workload(name: str, n_override: Optional[int] = None, sh_f32: bool = False):
    """Return (scene, cameras, meta) for a named workload.

    The BF16-SH workloads store bf16-rounded SH coefficients; sh_f32=True
    returns the FP32 draw instead (same seed, unrounded).

    tiny        2k Gaussians, 128x128, SH0, 16x16 tiles, FP32.
    single      200k Gaussians, 1296x840, SH3, FP32 (the single-view workload).
    sweep       1M Gaussians, 1600x1060, SH3 (list-length sweep, scales as drawn).
    sweep_half  the same scene with every scale multiplied by 0.5.
    batched     3M Gaussians, 8 orbit cameras at 2x486x324, 3x972x648, 3x1944x1296.
    diff        6M Gaussians, 4 cameras at 1920x1080.
    """
    meta = {"name": name, "tile": (16, 16), "sh_dtype": "f32"}
    if name == "tiny":
        scene, cams = tiny_scene(1, n_override or 2000)
        meta["target_seed"] = 101
        return scene, cams, meta
    if name == "single":
        scene = gmm_scene(2, n_override or 200_000)
        cams = orbit_cameras(np.random.default_rng(1002), [(1296, 840)])
        return scene, cams, meta
    if name in ("sweep", "sweep_half"):
        scene = gmm_scene(3, n_override or 1_000_000)
        if name == "sweep_half":
            scene.scales = (scene.scales * np.float32(0.5)).astype(np.float32)
        cams = orbit_cameras(np.random.default_rng(1003), [(1600, 1060)])
        return scene, cams, meta
    if name == "batched":
        scene = gmm_scene(4, n_override or 3_000_000)
        if not sh_f32:
            scene.sh = bf16_round(scene.sh)
        res = [(486, 324)] * 2 + [(972, 648)] * 3 + [(1944, 1296)] * 3
        cams = orbit_cameras(np.random.default_rng(1004), res)
        meta["sh_dtype"] = "bf16"
        return scene, cams, meta
    if name == "diff":
        scene = gmm_scene(5, n_override or 6_000_000)
        if not sh_f32:
            scene.sh = bf16_round(scene.sh)
        cams = orbit_cameras(np.random.default_rng(1005), [(1920, 1080)] * 4)
        meta["sh_dtype"] = "bf16"
        return scene, cams, meta
    raise ValueError(f"unknown workload {name!r}")
