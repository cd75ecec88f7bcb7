"""Seeded synthetic scenes and cameras.

This module only draws random numbers and builds cameras. It holds none of the
rendering arithmetic, so both the CPU oracle and the GPU path can take their
inputs from it without sharing any code of the method itself.

Scene parameters follow the Gaussian parameterisation of Speedy-Splat
(Sec. 3.1, the set G_i = {mu_i, s_i, r_i, h_i, sigma_i}): means [N,3],
scales [N,3] (linear, > 0), rotations [N,4] as unit quaternions (w, x, y, z),
opacities [N] in (0, 1) and spherical-harmonic coefficients [N, (d+1)^2, 3].
The pre-activation values (log-scales and opacity logits) are returned as well,
for the differentiable path.

Cameras are pinholes with x_cam = R x_world + t, +z forward, +x right, +y down,
and principal point at the image centre.

Every draw uses ``numpy.random.default_rng(seed)`` in the order
means, log-scales, quaternions, logits, SH.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Camera", "Scene", "look_at_camera", "orbit_cameras", "random_orbit_cameras",
    "scene_c0", "scene_c0_lowsigma", "scene_c1", "scene_c2", "scene_c3",
    "scene_c3_fd", "scene_c4", "scene_blobs", "fixture_scene", "camera_c0",
    "camera_c1", "cameras_c1", "cameras_c2", "camera_c3", "camera_fd",
    "C4_RESOLUTIONS", "request_stream",
]


@dataclass
class Camera:
    """Pinhole camera. All values are the FP32 numbers both renderers receive."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # [3,3] float32, world -> camera rotation (row-major)
    t: np.ndarray            # [3]   float32, world -> camera translation
    near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))
        self.near = float(np.float32(self.near))
        self.bg = tuple(float(np.float32(b)) for b in self.bg)

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    def with_size(self, width: int, height: int, fx: float | None = None):
        """Same pose, other resolution (focal scaled to keep the field of view)."""
        s = width / self.width
        f = self.fx * s if fx is None else fx
        return Camera(width, height, f, f, width / 2.0, height / 2.0, self.R, self.t,
                      self.near, self.bg)


@dataclass
class Scene:
    means: np.ndarray        # [N,3] f32
    scales: np.ndarray       # [N,3] f32, linear
    quats: np.ndarray        # [N,4] f32 (w,x,y,z), unit norm
    opacity: np.ndarray      # [N]   f32 in (0,1)
    sh: np.ndarray           # [N,K,3] f32
    log_scales: np.ndarray = field(default=None)
    logits: np.ndarray = field(default=None)
    sh_degree: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx].copy(), self.scales[idx].copy(), self.quats[idx].copy(),
                     self.opacity[idx].copy(), self.sh[idx].copy(),
                     None if self.log_scales is None else self.log_scales[idx].copy(),
                     None if self.logits is None else self.logits[idx].copy(),
                     self.sh_degree)


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _sigmoid32(x):
    x = np.asarray(x, dtype=np.float64)
    return _f32(1.0 / (1.0 + np.exp(-x)))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _finish(rng, means, log_s_mu, log_s_sd, logit_mu, logit_sd, sh_degree, dc_sd=0.5,
            rest_sd=0.2):
    n = means.shape[0]
    log_s = _f32(rng.normal(log_s_mu, log_s_sd, size=(n, 3)))
    quats = _f32(_unit_quats(rng, n))
    logits = _f32(rng.normal(logit_mu, logit_sd, size=n))
    k = (sh_degree + 1) ** 2
    sh = np.empty((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = rng.normal(0.0, dc_sd, size=(n, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, rest_sd, size=(n, k - 1, 3))
    return Scene(_f32(means), _f32(np.exp(log_s)), quats, _sigmoid32(logits), sh,
                 log_s, logits, sh_degree)


# ---------------------------------------------------------------- cameras

def look_at_camera(eye, target, width, height, fx, fy=None, up=(0.0, 1.0, 0.0),
                   near=0.2) -> Camera:
    """Camera at ``eye`` looking at ``target``; camera +y points away from ``up``."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    t = -R @ eye
    return Camera(width, height, fx, fx if fy is None else fy, width / 2.0, height / 2.0,
                  R, t, near)


def _hfov_focal(width, hfov_deg=60.0):
    return (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)


def orbit_cameras(k, radius, elevation_deg, width, height, hfov_deg=60.0):
    f = _hfov_focal(width, hfov_deg)
    cams = []
    for j in range(k):
        az = math.radians(360.0 * j / k)
        el = math.radians(elevation_deg)
        eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                 math.cos(el) * math.cos(az)])
        cams.append(look_at_camera(eye, (0.0, 0.0, 0.0), width, height, f))
    return cams


def random_orbit_cameras(rng, k, radius, width, height, el_range=(-15.0, 15.0),
                         hfov_deg=60.0):
    f = _hfov_focal(width, hfov_deg)
    cams = []
    for _ in range(k):
        az = math.radians(rng.uniform(0.0, 360.0))
        el = math.radians(rng.uniform(*el_range))
        eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                 math.cos(el) * math.cos(az)])
        cams.append(look_at_camera(eye, (0.0, 0.0, 0.0), width, height, f))
    return cams


def camera_c0() -> Camera:
    """256x256, fx = fy = 256, identity pose."""
    return Camera(256, 256, 256.0, 256.0, 128.0, 128.0, np.eye(3), np.zeros(3))


def camera_fd() -> Camera:
    """64x64, fx = fy = 64, identity pose (finite-difference subproblem)."""
    return Camera(64, 64, 64.0, 64.0, 32.0, 32.0, np.eye(3), np.zeros(3))


def cameras_c1(k=8):
    """1600x1040, 60 degree horizontal FOV, radius-12 orbit at 10 degrees elevation."""
    return orbit_cameras(k, 12.0, 10.0, 1600, 1040)


def camera_c1():
    return cameras_c1(8)[0]


def cameras_c2(k=64, seed=2):
    rng = np.random.default_rng(seed + 1000)
    return random_orbit_cameras(rng, k, 12.0, 1600, 1040)


def camera_c3():
    return orbit_cameras(8, 12.0, 10.0, 1264, 832)[1]


# ---------------------------------------------------------------- scenes

def scene_c0(n=10_000, seed=0, sh_degree=0, log_s=(-3.5, 0.5), logit=(0.0, 1.5)) -> Scene:
    """Uniform cube scene in front of an identity camera: x, y ~ U[-1,1], z ~ U[2,6]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(n, 3))
    means = np.stack([u[:, 0], u[:, 1], 4.0 + 2.0 * u[:, 2]], axis=1)
    return _finish(rng, means, log_s[0], log_s[1], logit[0], logit[1], sh_degree)


def scene_c0_lowsigma(n=10_000, seed=0) -> Scene:
    """The uniform cube scene with every opacity capped at 0.35."""
    s = scene_c0(n, seed)
    s.opacity = _f32(np.minimum(s.opacity, np.float32(0.35)))
    return s


def scene_blobs(n, seed, log_s=(-4.0, 1.0), logit=(0.0, 2.0), sh_degree=3, n_blobs=200,
                background=0.10) -> Scene:
    """Clustered scene: 200 anisotropic Gaussian blobs plus a uniform background
    in a 20-unit box."""
    rng = np.random.default_rng(seed)
    n_bg = int(round(n * background))
    n_fg = n - n_bg
    centres = rng.uniform(-8.0, 8.0, size=(n_blobs, 3))
    rot = _unit_quats(rng, n_blobs)
    ext = rng.uniform(0.2, 1.5, size=(n_blobs, 3))
    w, x, y, z = rot.T
    Rb = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)
    which = rng.integers(0, n_blobs, size=n_fg)
    local = rng.standard_normal((n_fg, 3)) * ext[which]
    fg = centres[which] + np.einsum("nij,nj->ni", Rb[which], local)
    bg = rng.uniform(-10.0, 10.0, size=(n_bg, 3))
    means = np.concatenate([fg, bg], axis=0)
    return _finish(rng, means, log_s[0], log_s[1], logit[0], logit[1], sh_degree)


def scene_c1(n=1_500_000, seed=1) -> Scene:
    return scene_blobs(n, seed)


def scene_c2(n=150_000, seed=2) -> Scene:
    return scene_blobs(n, seed, log_s=(-3.0, 1.0), logit=(1.0, 1.5))


def scene_c3(n=1_000_000, seed=3) -> Scene:
    return scene_blobs(n, seed)


def scene_c3_fd(n=2_000, seed=3) -> Scene:
    """Small SH-3 cube scene for finite-difference gradient checks (64x64 camera)."""
    return scene_c0(n, seed, sh_degree=3, log_s=(-2.5, 0.5))


C4_SCENE_SIZES = (300_000, 1_000_000, 3_000_000, 6_000_000)
C4_RESOLUTIONS = ((640, 480), (1280, 720), (1600, 1040), (1920, 1080))


def scene_c4(which: int, scale: float = 1.0) -> Scene:
    n = max(1, int(C4_SCENE_SIZES[which] * scale))
    return scene_blobs(n, 40 + which)


def request_stream(n_requests, qps, n_scenes=4, seed=44, resolutions=C4_RESOLUTIONS):
    """Poisson arrivals with a random scene, resolution and orbit camera per request.
    Returns a list of (arrival_s, scene_index, Camera)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arrivals = np.cumsum(gaps)
    out = []
    for k in range(n_requests):
        sidx = int(rng.integers(0, n_scenes))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        cam = random_orbit_cameras(rng, 1, 12.0, w, h)[0]
        out.append((float(arrivals[k]), sidx, cam))
    return out


# ---------------------------------------------------------------- fixtures

def fixture_scene(means, scales, quats, opacity, colours) -> Scene:
    """Hand-built scene from explicit per-Gaussian values (SH degree 0).
    ``colours`` are the DC coefficients."""
    means = _f32(np.atleast_2d(means))
    n = means.shape[0]
    sh = _f32(np.asarray(colours, dtype=np.float64).reshape(n, 1, 3))
    q = np.asarray(quats, dtype=np.float64).reshape(n, 4)
    return Scene(means, _f32(np.asarray(scales).reshape(n, 3)), _f32(q),
                 _f32(np.asarray(opacity).reshape(n)), sh, None, None, 0)
