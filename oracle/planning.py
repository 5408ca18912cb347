"""FP64 oracle of candidate-view generation and the overall exploration
criterion (Sec. 3.2: Eq. 5, Eq. 6, Eq. 7, "Exploration Strategy").

TEST INFRASTRUCTURE ONLY: the tests use this module; the product package
never does.  Plain numpy in float64, written from the definitions below.

Exploration map: an occupancy grid of nx * ny * nz voxels of edge `voxel`
starting at `origin`, one byte per voxel, x fastest; a byte of 1 marks an
observed free voxel.  Newly observed voxels are free now and were not free
in the previous grid.

Candidate positions: the centres of newly observed voxels on a lattice of
spacing s = round(step / voxel) voxels: ix and iy multiples of s, and iz on
the layers i0, i0 + s, ... of the voxel centres whose height lies in
[z_min - voxel/2, z_max + voxel/2) (i0 the first such layer; a single layer
when z_min == z_max).  Order: z, then y, then x (x fastest).

Viewing directions: the n points of the Fibonacci lattice on the unit
sphere, z_j = 1 - (2j + 1)/n, r_j = sqrt(1 - z_j^2), phi_j = j pi (3 - sqrt 5),
d_j = (r_j cos phi_j, r_j sin phi_j, z_j).  Candidate v = (position i,
direction j) with v = i n + j.

Camera of a candidate: world-to-camera rotation with rows (right, down,
forward) = (r, f x r, f), f = d_j, r = f x u / |f x u|, u = +z (or +x when
|f . z| > 0.99); t = -R p.  Stored as float32.

Overall criterion (Eq. 7) over the candidate pool, all softmaxes across the
candidates:
    I_geo  = softmax(log N_S)     = N_S / sum N_S          (Eq. 5)
    I_sem  = softmax(sum_p H)                               (Eq. 6)
    I      = (1 - softmax(l)) I_geo I_sem,  l = |T^v - T^t|  (Eq. 7)
A candidate with N_S < prune_fraction * pixels is pruned; the best
candidate is the unpruned one with the largest I (the first on ties), -1 if
none.  Readings: the softmaxes are taken over the whole pool before pruning;
if every N_S is 0, I_geo is 0 for all.
"""
from __future__ import annotations

import numpy as np


def fibonacci_directions(n: int) -> np.ndarray:
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = j * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def lattice_layers(nz: int, voxel: float, origin_z: float, step: float, z_min: float, z_max: float) -> list:
    s = max(1, int(round(step / voxel)))
    zc = origin_z + (np.arange(nz) + 0.5) * voxel
    inside = np.nonzero((zc >= z_min - 0.5 * voxel) & (zc < z_max + 0.5 * voxel))[0]
    if inside.size == 0:
        return []
    return list(range(int(inside[0]), int(inside[-1]) + 1, s))


def candidate_sites(free_now: np.ndarray, free_before: np.ndarray, dims, voxel: float, origin, step: float,
                    z_min: float, z_max: float) -> np.ndarray:
    """Positions [M, 3] (float64) of the candidate sites, in z, y, x order.
    free_now / free_before: flat uint8 arrays of nx*ny*nz (x fastest)."""
    nx, ny, nz = dims
    s = max(1, int(round(step / voxel)))
    fn = np.asarray(free_now).reshape(nz, ny, nx)
    fb = np.asarray(free_before).reshape(nz, ny, nx)
    out = []
    for iz in lattice_layers(nz, voxel, origin[2], step, z_min, z_max):
        for iy in range(0, ny, s):
            for ix in range(0, nx, s):
                if fn[iz, iy, ix] == 1 and fb[iz, iy, ix] != 1:
                    out.append([origin[0] + (ix + 0.5) * voxel, origin[1] + (iy + 0.5) * voxel,
                                origin[2] + (iz + 0.5) * voxel])
    return np.asarray(out, np.float64).reshape(-1, 3)


def pose(position, direction) -> np.ndarray:
    """12 floats: R row-major (world to camera) then t, float32."""
    f = np.asarray(direction, np.float64)
    f = f / np.linalg.norm(f)
    u = np.array([0.0, 0.0, 1.0])
    if abs(f[2]) > 0.99:
        u = np.array([1.0, 0.0, 0.0])
    r = np.cross(f, u)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ np.asarray(position, np.float64)
    return np.concatenate([R.reshape(-1), t]).astype(np.float32)


def candidates(free_now, free_before, dims, voxel, origin, step, directions, z_min, z_max):
    """(poses [V, 12] float32, positions [V, 3] float32), v = site * n + j."""
    sites = candidate_sites(free_now, free_before, dims, voxel, origin, step, z_min, z_max)
    dirs = fibonacci_directions(directions)
    poses = np.asarray([pose(p, d) for p in sites for d in dirs], np.float32).reshape(-1, 12)
    pos = np.repeat(sites, directions, axis=0).astype(np.float32)
    return poses, pos


def _softmax(x: np.ndarray) -> np.ndarray:
    m = np.max(x)
    e = np.exp(x - m)
    return e / e.sum()


def combine(n_empty, entropy_sum, positions, current, pixels, prune_fraction=0.005):
    """Eq. 5-7 over the pool.  Returns (score [V], pruned [V] bool, best)."""
    n = np.asarray(n_empty, np.float64)
    h = np.asarray(entropy_sum, np.float64)
    pos = np.asarray(positions, np.float64)
    tot = n.sum()
    i_geo = n / tot if tot > 0 else np.zeros_like(n)
    i_sem = _softmax(h)
    dist = np.sqrt(((pos - np.asarray(current, np.float64)) ** 2).sum(-1))
    score = (1.0 - _softmax(dist)) * i_geo * i_sem
    pruned = n < prune_fraction * np.asarray(pixels, np.float64)
    cand = np.nonzero(~pruned)[0]
    best = int(cand[np.argmax(score[cand])]) if cand.size else -1
    return score, pruned, best
