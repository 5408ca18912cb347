"""Next-best-view planning step over the C ABI (Sec. 3.2).

`Planner.step` runs, on the current stream:

1. sgr_generate_candidates: candidate poses from the newly observed voxels
   of the exploration map (one sampling stage: coarse or fine);
2. sgr_score_poses: the batched persistent scorer over those poses (empty
   pixels and summed entropy per view, Eq. 4-6), reading the poses straight
   from device memory;
3. sgr_combine_scores: the overall criterion with motion cost (Eq. 7),
   pruning, and the best candidate.

Host round trips: the candidate count after step 1, which sizes the
scoring launches, and a status read after each scoring launch of at most
`chunk` views (it grows the key capacity when needed).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L
from .rasterizer import Gaussians, _ptr

COARSE = dict(step=1.0, directions=5)   # one height plane
FINE = dict(step=0.5, directions=15)    # several heights


@dataclass
class Grid:
    """Exploration map geometry: dims (nx, ny, nz), voxel edge, origin."""
    dims: tuple
    voxel: float
    origin: tuple

    def c_struct(self) -> L.sgr_grid:
        nx, ny, nz = self.dims
        return L.sgr_grid(int(nx), int(ny), int(nz), float(self.voxel), (ctypes.c_float * 3)(*self.origin))


def sampling(step: float, directions: int, z_min: float, z_max: float) -> L.sgr_sampling:
    return L.sgr_sampling(float(step), int(directions), float(z_min), float(z_max))


class Planner:
    """Holds the device buffers of a planning step for one grid, image size
    and config; buffers grow with the candidate count."""

    def __init__(self, grid: Grid, intrinsics, cfg: L.sgr_config, capacity: int = 4096, device="cuda",
                 chunk: int = 128):
        self.grid = grid
        self.cfg = cfg
        self.device = torch.device(device)
        self.intr = (L.sgr_camera * 1)()
        c = intrinsics
        self.intr[0] = L.sgr_camera((ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1), (ctypes.c_float * 3)(0, 0, 0),
                                    float(c.fx), float(c.fy), float(c.cx), float(c.cy), int(c.width), int(c.height))
        self.pixels = int(c.width) * int(c.height)
        self.chunk = int(chunk)  # views per scoring launch: bounds the per-(view, Gaussian) workspace
        self.count = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.key_capacity = 0
        self._grow(capacity)
        self.cand_ws = None
        self.score_ws = None

    def _grow(self, capacity: int):
        self.capacity = int(capacity)
        dev = self.device
        self.poses = torch.empty((self.capacity, 12), dtype=torch.float32, device=dev)
        self.positions = torch.empty((self.capacity, 3), dtype=torch.float32, device=dev)
        self.n_empty = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.entropy = torch.empty(self.capacity, dtype=torch.float64, device=dev)
        self.score = torch.empty(self.capacity, dtype=torch.float64, device=dev)
        self.pruned = torch.empty(self.capacity, dtype=torch.uint8, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev)

    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def generate(self, free_now: torch.Tensor, free_before: torch.Tensor | None, samp: L.sgr_sampling) -> int:
        """Candidate poses into self.poses / self.positions; returns V."""
        gs = self.grid.c_struct()
        need = L.sgr_candidates_workspace_size(gs, samp)
        if need == 0:
            raise L.SgrError(L.SGR_EINVAL, "sgr_candidates_workspace_size")
        if self.cand_ws is None or self.cand_ws.numel() < need:
            self.cand_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        for _ in range(2):
            L.check(L.sgr_generate_candidates(gs, _ptr(free_now), _ptr(free_before), samp, self.capacity,
                                              _ptr(self.poses), _ptr(self.positions), _ptr(self.count),
                                              _ptr(self.cand_ws), self.cand_ws.numel(), self.stream),
                    "sgr_generate_candidates")
            V = int(self.count.item())
            if V <= self.capacity:
                return V
            self._grow(V)
        return V

    def score_views(self, g: Gaussians, V: int):
        """Empty-pixel counts and entropy sums of the first V candidates, in
        launches of at most `chunk` views."""
        for v0 in range(0, V, self.chunk):
            self._score_chunk(g, v0, min(self.chunk, V - v0))
        return self.n_empty[:V], self.entropy[:V]

    def _score_chunk(self, g: Gaussians, v0: int, nv: int):
        cams = self.intr
        for _ in range(3):
            cap = self.key_capacity or max(1 << 16, 4 * g.n)
            size = L.sgr_workspace_size(g.n, _repeat(cams, nv), nv, self.cfg, cap)
            if size == 0:
                raise L.SgrError(L.SGR_EINVAL, "sgr_workspace_size")
            if self.score_ws is None or self.score_ws.numel() < size:
                self.score_ws = torch.empty(size, dtype=torch.uint8, device=self.device)
            L.check(L.sgr_score_poses(g.c_struct(), cams, nv, _ptr(self.poses[v0:]), self.cfg, cap,
                                      _ptr(self.n_empty[v0:]), _ptr(self.entropy[v0:]), _ptr(self.score_ws),
                                      self.score_ws.numel(), self.stream), "sgr_score_poses")
            st, _, nk = L.sgr_read_status(_ptr(self.score_ws), self.stream)
            if st == L.SGR_ECAPACITY:
                self.key_capacity = int(nk * 1.25) + 4096
                continue
            L.check(st, "device status")
            self.key_capacity = cap
            return
        raise L.SgrError(L.SGR_ECAPACITY, "sgr_score_poses")

    def combine(self, V: int, current, prune_fraction: float = 0.005):
        L.check(L.sgr_combine_scores(V, _ptr(self.n_empty), _ptr(self.entropy), _ptr(self.positions), current,
                                     self.pixels, float(prune_fraction), _ptr(self.score), _ptr(self.pruned),
                                     _ptr(self.best), self.stream), "sgr_combine_scores")
        return self.score[:V], self.pruned[:V], self.best

    def step(self, g: Gaussians, free_now, free_before, samp: L.sgr_sampling, current, prune_fraction=0.005):
        """One planning step; returns a dict of device tensors (V may be 0)."""
        V = self.generate(free_now, free_before, samp)
        out = {"V": V}
        if V == 0:
            return out
        ne, hs = self.score_views(g, V)
        sc, pr, best = self.combine(V, current, prune_fraction)
        out.update(poses=self.poses[:V], positions=self.positions[:V], n_empty=ne, entropy_sum=hs, score=sc,
                   pruned=pr, best=best)
        return out


def _repeat(cams, V: int):
    """V copies of one sgr_camera (only the sizes matter for the workspace)."""
    arr = (L.sgr_camera * V)()
    for i in range(V):
        arr[i] = cams[0]
    return arr
