"""Seeded synthetic scenes and cameras.

This module only draws inputs: Gaussian parameters, cameras and targets.  It
holds none of the rasterizer's arithmetic, and both the HIP library's tests
and the FP64 oracle consume the same float32 arrays it returns.

The workloads stand in for the paper's Replica / Matterport3D rooms, which
are not available: a room-sized volume filled with small anisotropic
Gaussians, 1200x680 keyframes (Sec. 4.1 gives 680x1200 frames with a 90
degree horizontal field of view), top-16 sparse semantics over 102 classes
(Replica's 101 + unknown, Sec. 4.1 / supplement) or 40 classes (MP3D), and
candidate views on a Fibonacci sphere around a point (Sec. 3.2 samples view
directions on a Fibonacci lattice).

Draw order is fixed: means, scales, quaternions, opacity pre-activation,
rgb, semantic indices, semantic values, cameras, targets; generator PCG64
(numpy.random.default_rng(seed)).
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

_CHUNK = 65536


def generator_sha() -> str:
    with open(os.path.abspath(__file__), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


@dataclass
class Camera:
    """Pinhole camera, world->camera rotation R (row-major 3x3) and t.

    Camera axes follow OpenCV: x right, y down, z forward.  Pixel (col, row)
    has its centre at (col + 0.5, row + 0.5).
    """

    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclass
class Scene:
    means: np.ndarray  # f32 [N,3]
    scales: np.ndarray  # f32 [N,3], linear metres
    quats: np.ndarray  # f32 [N,4], (w,x,y,z)
    opacity: np.ndarray  # f32 [N], post-activation, in (0,1)
    rgb: np.ndarray  # f32 [N,3]
    sem_val: np.ndarray  # f32 [N,k]
    sem_idx: np.ndarray  # u8  [N,k]
    num_classes: int
    cameras: list = field(default_factory=list)
    candidates: list = field(default_factory=list)
    targets: dict = field(default_factory=dict)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def k(self) -> int:
        return int(self.sem_val.shape[1])


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _sem_indices(rng, n, c, k):
    out = np.empty((n, k), dtype=np.uint8)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = np.argsort(rng.random((e - s, c)), axis=1)[:, :k].astype(np.uint8)
    return out


def _sem_values(rng, n, k):
    d = rng.dirichlet(np.ones(k), size=n)
    d = -np.sort(-d, axis=1)
    v = d.astype(np.float32)
    return (v / v.sum(axis=1, dtype=np.float32, keepdims=True)).astype(np.float32)


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _room_gaussians(rng, n, box, c, k):
    lo = np.array([0.0, 0.0, 0.0])
    hi = np.asarray(box, dtype=np.float64)
    means = (lo + rng.random((n, 3)) * (hi - lo)).astype(np.float32)
    scales = np.exp(rng.normal(math.log(0.02), 0.5, size=(n, 3))).astype(np.float32)
    quats = _unit_quats(rng, n).astype(np.float32)
    opacity = _sigmoid(rng.normal(0.0, 1.5, size=n)).astype(np.float32)
    rgb = rng.random((n, 3)).astype(np.float32)
    sem_idx = _sem_indices(rng, n, c, k)
    sem_val = _sem_values(rng, n, k)
    return means, scales, quats, opacity, rgb, sem_val, sem_idx


def look_at(pos, target, width, height, fx, fy, cx=None, cy=None, up=(0.0, 0.0, 1.0)) -> Camera:
    pos = np.asarray(pos, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - pos
    f /= np.linalg.norm(f)
    upv = np.asarray(up, dtype=np.float64)
    if abs(float(f @ upv)) > 0.99:
        upv = np.array([1.0, 0.0, 0.0])
    r = np.cross(f, upv)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ pos)).astype(np.float32)
    return Camera(R, t, float(fx), float(fy), float(width / 2 if cx is None else cx),
                  float(height / 2 if cy is None else cy), int(width), int(height))


def fibonacci_sphere(n: int) -> np.ndarray:
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - 2.0 * (j + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _quat_rot(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


_SIZES = ((160, 120), (320, 240), (640, 480))


def sphere_candidates(rng, nviews, box_lo, box_hi, radius=1.5, sizes=_SIZES):
    """Poses on a radius-1.5 m Fibonacci sphere around a random centre,
    looking at the centre, each with a resolution drawn from `sizes`
    (fx = fy = W/2, i.e. a 90 degree horizontal field of view)."""
    c = np.asarray(box_lo) + rng.random(3) * (np.asarray(box_hi) - np.asarray(box_lo))
    rot = _quat_rot(_unit_quats(rng, 1)[0])
    u = fibonacci_sphere(nviews) @ rot.T
    pick = rng.integers(0, len(sizes), size=nviews)
    cams = []
    for j in range(nviews):
        w, h = sizes[int(pick[j])]
        cams.append(look_at(c + radius * u[j], c, w, h, w / 2, w / 2))
    return cams


def room_view_camera():
    """1200x680 keyframe at the room centre (5, 4, 1.5) looking along +x."""
    R = np.array([[0, -1, 0], [0, 0, -1], [1, 0, 0]], dtype=np.float32)
    c = np.array([5.0, 4.0, 1.5])
    t = (-(R.astype(np.float64) @ c)).astype(np.float32)
    return Camera(R, t, 600.0, 600.0, 600.0, 340.0, 1200, 680)


def l1_targets(rng, cam: Camera, num_classes: int):
    h, w = cam.height, cam.width
    return {
        "rgb": rng.random((h, w, 3)).astype(np.float32),
        "depth": rng.uniform(0.5, 5.0, size=(h, w)).astype(np.float32),
        "label": rng.integers(0, num_classes, size=(h, w)).astype(np.int32),
    }


def tiny_scene(seed=0, n=2000, num_classes=16, k=3, width=64, height=64, f=60.0) -> Scene:
    """2000 Gaussians 1-3 m in front of a 64x64 identity-pose camera,
    isotropic log-normal scales (mean log 0.03 m, sigma 0.3), identity
    rotations, top-3 of 16 classes."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(1, 3, n)], 1).astype(np.float32)
    s = np.exp(rng.normal(math.log(0.03), 0.3, size=n))
    scales = np.repeat(s[:, None], 3, axis=1).astype(np.float32)
    quats = np.tile(np.array([1, 0, 0, 0], dtype=np.float32), (n, 1))
    opacity = _sigmoid(rng.normal(0.0, 1.5, size=n)).astype(np.float32)
    rgb = rng.random((n, 3)).astype(np.float32)
    sem_idx = _sem_indices(rng, n, num_classes, k)
    sem_val = _sem_values(rng, n, k)
    cam = Camera(np.eye(3, dtype=np.float32), np.zeros(3, dtype=np.float32), f, f,
                 width / 2, height / 2, width, height)
    return Scene(means, scales, quats, opacity, rgb, sem_val, sem_idx, num_classes, [cam], name="tiny64")


def room_scene(seed=0, n=200_000, num_classes=102, k=16, targets=True) -> Scene:
    """n Gaussians uniform in a 10x8x3 m room, anisotropic log-normal scales
    (mean log 0.02 m, sigma 0.5), random unit quaternions, top-16 of 102
    classes; one 1200x680 keyframe (fx=fy=600) and seeded L1 targets."""
    rng = np.random.default_rng(seed)
    g = _room_gaussians(rng, n, (10.0, 8.0, 3.0), num_classes, k)
    cam = room_view_camera()
    sc = Scene(*g, num_classes, [cam], name=f"room{n}")
    if targets:
        sc.targets = l1_targets(rng, cam, num_classes)
    return sc


def candidate_scene(seed=0, n=500_000, nviews=64, num_classes=102, k=16) -> Scene:
    """n Gaussians (room distributions) and nviews candidate poses of mixed
    resolution {160x120, 320x240, 640x480} on a 1.5 m sphere."""
    rng = np.random.default_rng(seed)
    g = _room_gaussians(rng, n, (10.0, 8.0, 3.0), num_classes, k)
    cams = sphere_candidates(rng, nviews, (1.5, 1.5, 0.5), (8.5, 6.5, 2.5))
    return Scene(*g, num_classes, cams, name=f"cand{n}x{nviews}")


def large_scene(seed=0, n=3_000_000, nkey=8, ncand=128, num_classes=40, k=16) -> Scene:
    """n Gaussians in a 20x15x3 m multi-room volume, top-16 of 40 classes;
    nkey 1024x1280 keyframes (fx=fy=640) with random yaw and +-15 degree
    pitch, plus ncand 320x240 candidates on a sphere."""
    rng = np.random.default_rng(seed)
    g = _room_gaussians(rng, n, (20.0, 15.0, 3.0), num_classes, k)
    keys = []
    for _ in range(nkey):
        pos = np.array([rng.uniform(2, 18), rng.uniform(2, 13), rng.uniform(1.2, 1.8)])
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-15, 15))
        fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
        keys.append(look_at(pos, pos + fwd, 1024, 1280, 640, 640, 512, 640))
    cands = sphere_candidates(rng, ncand, (2.0, 2.0, 0.5), (18.0, 13.0, 2.5), sizes=((320, 240),))
    sc = Scene(*g, num_classes, keys, name=f"large{n}")
    sc.candidates = cands
    return sc
