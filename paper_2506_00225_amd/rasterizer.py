"""Torch-facing layer over libsgr: device memory and streams come from
PyTorch, every step of the rasterizer runs in the HIP library.

    frame = Frame(n, cameras, make_config(C, k))
    maps = render(gaussians, frame)                 # autograd-aware
    n_empty, entropy = frame.score(gaussians)       # candidate-view scoring
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

DEFAULTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, z_near=0.2, lowpass=0.3)


def make_config(num_classes: int, top_k: int, sem_grad_to_geometry: int = 0, sem_accumulators: int = 0,
                tile_order: int = 0, score_workgroups: int = 0, sem_passes: int = 0, bwd_batch: int = 0,
                radix_bits: int = 0, **kw) -> L.sgr_config:
    """sem_accumulators (0 automatic, 1 LDS, 2 registers for C <= 128),
    tile_order (0 automatic, 1 XCD-contiguous, 2 linear),
    score_workgroups (0 = all resident), sem_passes (0 automatic, 1..4
    class ranges of the LDS class sums), bwd_batch (0 = 44, or 32, 44, 56
    keys per backward batch) and radix_bits (0 = 8, or 6 or 8 bits per
    sort pass) change speed only, not the bits of any output (see autotune)."""
    d = dict(DEFAULTS)
    d.update(kw)
    return L.sgr_config(d["alpha_min"], d["alpha_max"], d["t_min"], d["z_near"], d["lowpass"], int(num_classes),
                        int(top_k), int(sem_grad_to_geometry), 16, 16, int(sem_accumulators), int(tile_order),
                        int(score_workgroups), int(sem_passes), int(bwd_batch), int(radix_bits))


def camera_array(cams):
    arr = (L.sgr_camera * len(cams))()
    for j, c in enumerate(cams):
        R = [float(x) for x in c.R.reshape(-1)]
        t = [float(x) for x in c.t.reshape(-1)]
        arr[j] = L.sgr_camera((ctypes.c_float * 9)(*R), (ctypes.c_float * 3)(*t), c.fx, c.fy, c.cx, c.cy,
                              int(c.width), int(c.height))
    return arr


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _device(device) -> torch.device:
    """torch.device with the index filled in ("cuda" means the current
    device), so it compares equal to a tensor's device."""
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device() if torch.cuda.is_available() else 0)
    return d


@dataclass
class Gaussians:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacity: torch.Tensor
    rgb: torch.Tensor
    sem_val: torch.Tensor
    sem_idx: torch.Tensor  # uint8

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def k(self) -> int:
        return int(self.sem_val.shape[1])

    def validate(self, n: int | None = None, k: int | None = None, device=None):
        """Raises ValueError unless every tensor is contiguous, on one CUDA
        device, of the right dtype and of shape means/scales/rgb [n, 3],
        quats [n, 4], opacity [n], sem_val/sem_idx [n, k] (n and k from the
        means and sem_val unless given: a Frame passes its own)."""
        n = self.n if n is None else int(n)
        k = self.k if k is None else int(k)
        dev = self.means.device if device is None else _device(device)
        shapes = {"means": (n, 3), "scales": (n, 3), "quats": (n, 4), "opacity": (n,), "rgb": (n, 3),
                  "sem_val": (n, k), "sem_idx": (n, k)}
        for name, shape in shapes.items():
            t = getattr(self, name)
            want = torch.uint8 if name == "sem_idx" else torch.float32
            if not isinstance(t, torch.Tensor) or t.dtype != want:
                raise ValueError(f"{name}: need a {want} tensor")
            if tuple(t.shape) != shape:
                raise ValueError(f"{name}: shape {tuple(t.shape)}, need {shape}")
            if not t.is_contiguous():
                raise ValueError(f"{name}: need a contiguous tensor")
        for name in shapes:
            t = getattr(self, name)
            if not t.is_cuda or t.device != dev:
                raise ValueError(f"{name}: need a CUDA tensor on {dev}")

    def c_struct(self, frame: "Frame | None" = None) -> L.sgr_gaussians:
        if frame is None:
            self.validate()
        else:
            self.validate(frame.n, frame.cfg.top_k, frame.device)
        return L.sgr_gaussians(self.n, _ptr(self.means), _ptr(self.scales), _ptr(self.quats), _ptr(self.opacity),
                               _ptr(self.rgb), _ptr(self.sem_val), _ptr(self.sem_idx))

    @staticmethod
    def from_scene(scene, device="cuda") -> "Gaussians":
        f = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float32).contiguous()
        return Gaussians(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacity), f(scene.rgb),
                         f(scene.sem_val), torch.from_numpy(scene.sem_idx).to(device).contiguous())


class Frame:
    """Cameras, config and the library workspace for one batch of views."""

    def __init__(self, n: int, cams, cfg: L.sgr_config, key_capacity: int | None = None, device="cuda"):
        L.lib()
        self.n = int(n)
        self.cam_list = list(cams)
        self.cams = camera_array(self.cam_list)
        self.V = len(self.cam_list)
        self.cfg = cfg
        self.device = _device(device)
        self.sizes = [(int(c.height), int(c.width)) for c in self.cam_list]
        self.pix = [h * w for h, w in self.sizes]
        self.pix_off = [0]
        for p in self.pix:
            self.pix_off.append(self.pix_off[-1] + p)
        self.key_capacity = int(key_capacity or max(1 << 16, 2 * self.n * self.V))
        # bumped by every call that rewrites the workspace state a backward
        # reads (projection, sort, per-pixel transmittance and last index)
        self.generation = 0
        self._alloc()

    def _alloc(self):
        size = L.sgr_workspace_size(self.n, self.cams, self.V, self.cfg, self.key_capacity)
        if size == 0:
            raise L.SgrError(L.SGR_EINVAL, "sgr_workspace_size")
        self.ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.layout = L.sgr_workspace_layout(self.n, self.cams, self.V, self.cfg, self.key_capacity)

    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _args(self):
        return (self.cams, self.V, self.cfg, self.key_capacity)

    # ------------------------------------------------------------ pipeline steps

    def project(self, g: Gaussians):
        self.generation += 1
        L.check(L.sgr_project(g.c_struct(self), *self._args(), _ptr(self.ws), self.ws.numel(), self.stream),
                "sgr_project")

    def bin(self, g: Gaussians, d_num_keys=None):
        self.generation += 1
        if d_num_keys is not None:
            self._check_tensor("d_num_keys", d_num_keys, torch.int64, 1)
        L.check(L.sgr_bin(g.c_struct(self), *self._args(), _ptr(d_num_keys), _ptr(self.ws), self.ws.numel(),
                          self.stream), "sgr_bin")

    def status(self):
        """(status, visible pairs, keys); synchronises the stream."""
        return L.sgr_read_status(_ptr(self.ws), self.stream)

    def prepare(self, g: Gaussians, check: bool = True):
        """project + bin; with check, grows the key capacity when exceeded."""
        for _ in range(3):
            self.project(g)
            self.bin(g)
            if not check:
                return
            st, _, nk = self.status()
            if st == L.SGR_ECAPACITY:
                self.key_capacity = int(nk * 1.25) + 1024
                self._alloc()
                continue
            L.check(st, "device status")
            return
        raise L.SgrError(L.SGR_ECAPACITY, "prepare")

    def alloc_maps(self, want=("rgb", "depth", "sil", "sem")):
        P = self.pix_off[-1]
        C = self.cfg.num_classes
        dev = self.device
        maps = {
            "rgb": torch.empty((P, 3), device=dev) if "rgb" in want else None,
            "depth": torch.empty(P, device=dev) if "depth" in want else None,
            "sil": torch.empty(P, device=dev) if "sil" in want else None,
            "sem": torch.empty((P, C), device=dev) if "sem" in want else None,
            "t_final": torch.empty(P, device=dev),
            "n_contrib": torch.empty(P, dtype=torch.int32, device=dev),
        }
        return maps

    def _check_tensor(self, name, t, dtype, numel):
        if not isinstance(t, torch.Tensor) or t.dtype != dtype:
            raise ValueError(f"{name}: need a {dtype} tensor")
        if t.numel() < numel:
            raise ValueError(f"{name}: {t.numel()} elements, need {numel}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous tensor")
        if not t.is_cuda or t.device != self.device:
            raise ValueError(f"{name}: need a CUDA tensor on {self.device}")

    def _view_ptrs(self, flat, ch, elem, name="map", dtype=torch.float32):
        """Per-view pointers into a flat [sum HW, ch] tensor (checked first)."""
        if flat is None:
            return [None] * self.V
        self._check_tensor(name, flat, dtype, self.pix_off[-1] * ch)
        base = flat.data_ptr()
        return [ctypes.c_void_p(base + self.pix_off[v] * ch * elem) for v in range(self.V)]

    def _map_table(self, maps):
        C = self.cfg.num_classes
        cols = {"rgb": 3, "depth": 1, "sil": 1, "sem": C, "t_final": 1, "n_contrib": 1}
        ptrs = {key: self._view_ptrs(maps.get(key), cols[key], 4, name=key,
                                     dtype=torch.int32 if key == "n_contrib" else torch.float32) for key in cols}
        arr = (L.sgr_maps * self.V)()
        for v in range(self.V):
            arr[v] = L.sgr_maps(ptrs["rgb"][v], ptrs["depth"][v], ptrs["sil"][v], ptrs["sem"][v],
                                ptrs["t_final"][v], ptrs["n_contrib"][v])
        return arr

    def forward(self, g: Gaussians, maps=None):
        maps = maps if maps is not None else self.alloc_maps()
        arr = self._map_table(maps)
        self.generation += 1
        L.check(L.sgr_render_forward(g.c_struct(self), *self._args(), arr, _ptr(self.ws), self.ws.numel(), self.stream),
                "sgr_render_forward")
        return maps

    def forward_dense(self, g: Gaussians, dense_sem: torch.Tensor, maps=None):
        """Forward with a dense [n, C] semantic distribution per Gaussian
        (all classes blended) instead of the top-k lists; after prepare()."""
        maps = maps if maps is not None else self.alloc_maps()
        dense_sem = dense_sem.to(device=self.device, dtype=torch.float32).contiguous()
        C = self.cfg.num_classes
        if dense_sem.shape != (self.n, C):
            raise ValueError(f"dense_sem must be [{self.n}, {C}]")
        arr = self._map_table(maps)
        self.generation += 1
        L.check(L.sgr_render_forward_dense(g.c_struct(self), _ptr(dense_sem), *self._args(), arr, _ptr(self.ws),
                                           self.ws.numel(), self.stream), "sgr_render_forward_dense")
        return maps

    def forward_loss(self, g: Gaussians, targets, loss_cfg=None, maps=None, grads=None, sparse_sem=False):
        """Forward render with the mapping loss fused into the same launch.

        targets: one dict per view (or one dict for a single view) with
        "rgb" [P,3], "depth" [P] and optionally "label" [P] (int32,
        cross-entropy) or "sem" [P,C] (pseudo-ground-truth distribution:
        entropy-masked Hellinger + cosine), all flat over the view's pixels.
        loss_cfg: an sgr_loss_config (loss_config() defaults if None).
        maps: optional dict of map tensors to write as well (any subset).
        Returns (grads, loss) with grads flat over all views like
        alloc_maps(), ready for backward(), and loss a float64 [V] tensor.
        With sparse_sem (cross-entropy targets), the semantic gradient comes
        back as "sem_label" / "sem_at_label", one class per pixel, instead
        of a dense [P, C] map."""
        targets = [targets] if isinstance(targets, dict) else list(targets)
        if len(targets) != self.V:
            raise ValueError("one target dict per view")
        C = self.cfg.num_classes
        dev = self.device
        P = self.pix_off[-1]
        if grads is None:
            grads = {"rgb": torch.empty((P, 3), device=dev), "depth": torch.empty(P, device=dev),
                     "sil": torch.empty(P, device=dev)}
            if sparse_sem:
                grads["sem_at_label"] = torch.empty(P, device=dev)
                grads["sem_label"] = torch.cat([
                    (t["label"].to(device=dev, dtype=torch.int32).reshape(-1) if t.get("label") is not None else
                     torch.full((self.pix[v],), -1, dtype=torch.int32, device=dev)) for v, t in enumerate(targets)])
            else:
                grads["sem"] = torch.empty((P, C), device=dev)
        cols = {"rgb": 3, "depth": 1, "sil": 1, "sem": C}
        arr = self._map_table(maps) if maps is not None else None
        gp = {key: self._view_ptrs(grads.get(key), cols[key], 4, name="grad " + key)
              for key in ("rgb", "depth", "sil", "sem")}
        gp["sem_at_label"] = self._view_ptrs(grads.get("sem_at_label"), 1, 4, name="grad sem_at_label")
        keep = []
        lv = (L.sgr_loss_view * self.V)()
        for v, t in enumerate(targets):
            tp = {}
            for key, dt, ch in (("rgb", torch.float32, 3), ("depth", torch.float32, 1), ("label", torch.int32, 1),
                                ("sem", torch.float32, C)):
                x = t.get(key)
                if x is not None:
                    x = x.to(device=dev, dtype=dt).contiguous()
                    if x.numel() != self.pix[v] * ch:
                        raise ValueError(f"target {key} of view {v}: {x.numel()} elements, need {self.pix[v] * ch}")
                    keep.append(x)
                tp[key] = _ptr(x)
            lv[v] = L.sgr_loss_view(tp["rgb"], tp["depth"], tp["label"], tp["sem"], gp["rgb"][v], gp["depth"][v],
                                    gp["sil"][v], gp["sem"][v], gp["sem_at_label"][v])
        loss = torch.empty(self.V, dtype=torch.float64, device=dev)
        lc = loss_cfg if loss_cfg is not None else loss_config()
        self.generation += 1
        L.check(L.sgr_render_forward_loss(g.c_struct(self), *self._args(), arr, lv, lc, _ptr(loss), _ptr(self.ws),
                                          self.ws.numel(), self.stream), "sgr_render_forward_loss")
        return grads, loss

    def _map_grads(self, grads: dict):
        """sgr_map_grads per view from flat tensors; "sem" is the dense
        [P, C] gradient, or "sem_label" [P] (int32) with "sem_at_label" [P]
        give it as one class per pixel."""
        C = self.cfg.num_classes
        cols = {"rgb": 3, "depth": 1, "sil": 1, "sem": C, "sem_label": 1, "sem_at_label": 1}
        gp = {}
        for key in cols:
            t = grads.get(key)
            if t is not None:
                want = torch.int32 if key == "sem_label" else torch.float32
                t = t.contiguous()
                if t.dtype != want:
                    t = t.to(want)
                grads[key] = t
            gp[key] = self._view_ptrs(t, cols[key], 4, name="grad " + key,
                                      dtype=torch.int32 if key == "sem_label" else torch.float32)
        arr = (L.sgr_map_grads * self.V)()
        for v in range(self.V):
            arr[v] = L.sgr_map_grads(gp["rgb"][v], gp["depth"][v], gp["sil"][v], gp["sem"][v], gp["sem_label"][v],
                                     gp["sem_at_label"][v])
        return arr

    @staticmethod
    def _grads(g: Gaussians, out: dict | None):
        names = ("means", "scales", "quats", "opacity", "rgb", "sem_val")
        if out is None:
            out = {name: torch.empty_like(getattr(g, name)) for name in names}
        for name in names:
            t, ref = out.get(name), getattr(g, name)
            if t is None:
                continue
            if (not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.shape != ref.shape
                    or t.device != ref.device or not t.is_contiguous()):
                raise ValueError(f"gradient {name}: need a contiguous float32 tensor of shape {tuple(ref.shape)} "
                                 f"on {ref.device}")
        gr = L.sgr_grads(*[_ptr(out[name]) for name in ("means", "scales", "quats", "opacity", "rgb", "sem_val")])
        return out, gr

    def backward(self, g: Gaussians, grads: dict, out: dict | None = None):
        arr = self._map_grads(grads)
        out, gr = self._grads(g, out)
        L.check(L.sgr_render_backward(g.c_struct(self), *self._args(), arr, gr, _ptr(self.ws), self.ws.numel(),
                                      self.stream), "sgr_render_backward")
        return out

    def backward_tiles(self, g: Gaussians, grads: dict):
        """First half of backward: per-key gradient slots (kept in the workspace)."""
        arr = self._map_grads(grads)
        L.check(L.sgr_render_backward_tiles(g.c_struct(self), *self._args(), arr, _ptr(self.ws), self.ws.numel(),
                                            self.stream), "sgr_render_backward_tiles")

    def backward_gather(self, g: Gaussians, out: dict | None = None):
        """Second half of backward: per-Gaussian gradients from the key slots."""
        out, gr = self._grads(g, out)
        L.check(L.sgr_render_backward_gather(g.c_struct(self), *self._args(), gr, _ptr(self.ws), self.ws.numel(),
                                             self.stream), "sgr_render_backward_gather")
        return out

    def backward_gather_adam(self, g: Gaussians, opt: "FusedAdam"):
        """backward_gather and opt.step() in one pass
        (sgr_render_backward_gather_adam): the gradients update the
        parameters where they are formed and are not written.  opt's six
        groups are the means, scales, quats, opacity, rgb and sem_val
        parameters, in this order (normally g's own tensors)."""
        n, k = self.n, int(self.cfg.top_k)
        want = (3 * n, 3 * n, 4 * n, n, 3 * n, k * n)
        if len(opt.groups) != 6 or any(p.numel() != w for (p, _, _, _), w in zip(opt.groups, want)):
            raise ValueError("backward_gather_adam: opt needs six groups (means, scales, quats, opacity, rgb, "
                             f"sem_val) of {want} elements")
        opt.t += 1
        L.check(L.sgr_render_backward_gather_adam(g.c_struct(self), *self._args(), opt.segs, opt.lr, opt.b1, opt.b2,
                                                  opt.eps, opt.t, _ptr(self.ws), self.ws.numel(), self.stream),
                "sgr_render_backward_gather_adam")

    def score(self, g: Gaussians, n_empty=None, entropy_sum=None):
        n_empty = n_empty if n_empty is not None else torch.empty(self.V, dtype=torch.int32, device=self.device)
        entropy_sum = entropy_sum if entropy_sum is not None else torch.empty(self.V, dtype=torch.float64,
                                                                                device=self.device)
        self._check_tensor("n_empty", n_empty, torch.int32, self.V)
        self._check_tensor("entropy_sum", entropy_sum, torch.float64, self.V)
        self.generation += 1
        L.check(L.sgr_score_views(g.c_struct(self), *self._args(), _ptr(n_empty), _ptr(entropy_sum), _ptr(self.ws),
                                  self.ws.numel(), self.stream), "sgr_score_views")
        return n_empty, entropy_sum

    def capture_score(self, g: Gaussians, n_empty=None, entropy_sum=None):
        """Captures sgr_score_views for these cameras into a HIP graph (every
        launch of the frame goes on the capture stream; camera tables travel
        as kernel arguments, so nothing is copied from the host).  Returns
        (graph, n_empty, entropy_sum); graph.replay() rescores the current
        contents of the Gaussian tensors."""
        n_empty = n_empty if n_empty is not None else torch.empty(self.V, dtype=torch.int32, device=self.device)
        entropy_sum = entropy_sum if entropy_sum is not None else torch.empty(self.V, dtype=torch.float64,
                                                                                device=self.device)
        self.score(g, n_empty, entropy_sum)  # warm-up outside capture (sets kernel attributes)
        torch.cuda.synchronize(self.device)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.score(g, n_empty, entropy_sum)
        return graph, n_empty, entropy_sum

    def split(self, flat):
        """Per-view [H, W, ...] views of a flat [sum HW, ...] tensor."""
        out = []
        for v, (h, w) in enumerate(self.sizes):
            t = flat[self.pix_off[v]:self.pix_off[v + 1]]
            out.append(t.reshape(h, w, *flat.shape[1:]))
        return out

    # ------------------------------------------------------------ inspection

    def workspace_u32(self, offset: int, count: int) -> torch.Tensor:
        return self.ws[offset:offset + 4 * count].view(torch.int32)


def score_maps(sem: torch.Tensor, n_contrib: torch.Tensor, num_classes: int, scratch: torch.Tensor | None = None,
               n_empty=None, entropy_sum=None):
    """Plain scoring of one dense view: sem [H, W, C], n_contrib [H, W]."""
    H, W = int(n_contrib.shape[0]), int(n_contrib.shape[1])
    need = L.sgr_score_maps_workspace_size(W, H)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=sem.device)
    n_empty = n_empty if n_empty is not None else torch.empty(1, dtype=torch.int32, device=sem.device)
    entropy_sum = entropy_sum if entropy_sum is not None else torch.empty(1, dtype=torch.float64, device=sem.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(sem.device).cuda_stream)
    L.check(L.sgr_score_maps(_ptr(sem), _ptr(n_contrib), W, H, int(num_classes), _ptr(n_empty), _ptr(entropy_sum),
                             _ptr(scratch), scratch.numel(), stream), "sgr_score_maps")
    return n_empty, entropy_sum


def score_maps_noalloc(sem: torch.Tensor, n_contrib: torch.Tensor, num_classes: int, n_empty: torch.Tensor,
                       entropy_sum: torch.Tensor):
    """score_maps without a workspace (sgr_score_maps_noalloc): the library
    allocates nothing, and neither does this wrapper; the caller passes
    n_empty (int32 [1]) and entropy_sum (float64 [1]) on sem's device.  At
    most L.SGR_NOALLOC_MAX_PIXELS pixels; calls that overlap on one GPU race
    on the library's static scratch."""
    H, W = int(n_contrib.shape[0]), int(n_contrib.shape[1])
    if W * H > L.SGR_NOALLOC_MAX_PIXELS:
        raise ValueError(f"{W}x{H} view: score_maps_noalloc takes at most {L.SGR_NOALLOC_MAX_PIXELS} pixels")
    for name, t, dt, numel in (("sem", sem, torch.float32, W * H * int(num_classes)),
                               ("n_contrib", n_contrib, torch.int32, W * H), ("n_empty", n_empty, torch.int32, 1),
                               ("entropy_sum", entropy_sum, torch.float64, 1)):
        if t.dtype != dt or not t.is_cuda or t.device != sem.device or not t.is_contiguous() or t.numel() < numel:
            raise ValueError(f"{name}: need a contiguous {dt} tensor of {numel} elements on {sem.device}")
    stream = ctypes.c_void_p(torch.cuda.current_stream(sem.device).cuda_stream)
    L.check(L.sgr_score_maps_noalloc(_ptr(sem), _ptr(n_contrib), W, H, int(num_classes), _ptr(n_empty),
                                     _ptr(entropy_sum), stream), "sgr_score_maps_noalloc")
    return n_empty, entropy_sum


class _Render(torch.autograd.Function):
    """The backward reads what the forward left in the frame's workspace
    (sorted keys, per-pixel final transmittance and last index): the frame's
    generation is recorded, and a backward after another call rewrote that
    state raises instead of returning wrong gradients.  The parameters are
    saved for backward, so autograd also rejects an in-place update made
    between the two."""

    @staticmethod
    def forward(ctx, frame, sem_idx, check, means, scales, quats, opacity, rgb, sem_val):
        g = Gaussians(means.detach(), scales.detach(), quats.detach(), opacity.detach(), rgb.detach(),
                      sem_val.detach(), sem_idx)
        frame.prepare(g, check=check)
        maps = frame.forward(g)
        ctx.frame = frame
        ctx.generation = frame.generation
        ctx.sem_idx = sem_idx
        ctx.save_for_backward(means, scales, quats, opacity, rgb, sem_val)
        ctx.mark_non_differentiable(maps["t_final"], maps["n_contrib"])
        return maps["rgb"], maps["depth"], maps["sil"], maps["sem"], maps["t_final"], maps["n_contrib"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_sil, g_sem, _gt, _gn):
        if ctx.frame.generation != ctx.generation:
            raise RuntimeError("render backward: the frame was used by another call (project, bin, forward or "
                               "score) after this render's forward; its workspace no longer holds this render")
        means, scales, quats, opacity, rgb, sem_val = ctx.saved_tensors
        g = Gaussians(means.detach(), scales.detach(), quats.detach(), opacity.detach(), rgb.detach(),
                      sem_val.detach(), ctx.sem_idx)
        grads = ctx.frame.backward(g, {"rgb": g_rgb, "depth": g_depth, "sil": g_sil, "sem": g_sem})
        return (None, None, None, grads["means"], grads["scales"], grads["quats"], grads["opacity"], grads["rgb"],
                grads["sem_val"])


def render(g: Gaussians, frame: Frame, check: bool = True):
    """Differentiable render of every view of `frame`.  Returns flat
    [sum HW, ...] tensors rgb, depth, sil, sem, t_final, n_contrib
    (frame.split gives per-view images)."""
    rgb, depth, sil, sem, t_final, n_contrib = _Render.apply(frame, g.sem_idx, check, g.means, g.scales, g.quats,
                                                             g.opacity, g.rgb, g.sem_val)
    return {"rgb": rgb, "depth": depth, "sil": sil, "sem": sem, "t_final": t_final, "n_contrib": n_contrib}


MAPPING_LOSS_WEIGHTS = (1.0, 0.5, 1.0, 1.0, 0.99)  # depth, colour, silhouette, cross-entropy, mask threshold


def loss_config(w_depth=1.0, w_rgb=0.5, w_sil=1.0, w_sem=1.0, sil_thresh=0.99, ce_floor=1e-6, lambda_hd=0.8,
                lambda_cos=0.2, entropy_tau=0.0, sqrt_eps=1e-8) -> L.sgr_loss_config:
    """Weights of the fused mapping loss (entropy_tau <= 0 means ln k)."""
    return L.sgr_loss_config(w_depth, w_rgb, w_sil, w_sem, sil_thresh, ce_floor, lambda_hd, lambda_cos, entropy_tau,
                             sqrt_eps)


def mapping_loss_grad(maps: dict, t_rgb, t_depth, label, num_classes: int, out: dict | None = None,
                      scratch=None, weights=MAPPING_LOSS_WEIGHTS):
    """dL/d(maps) of the mapping loss (see sgr_mapping_loss_grad); all flat
    [P, ...] tensors on one device."""
    P = int(maps["depth"].shape[0])
    dev = maps["depth"].device
    if out is None:
        out = {"rgb": torch.empty(P, 3, device=dev), "depth": torch.empty(P, device=dev),
               "sil": torch.empty(P, device=dev), "sem": torch.empty(P, num_classes, device=dev)}
    if scratch is None:
        scratch = torch.empty(P, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    L.check(L.sgr_mapping_loss_grad(_ptr(maps["rgb"]), _ptr(maps["depth"]), _ptr(maps["sil"]), _ptr(maps["sem"]),
                                    _ptr(t_rgb), _ptr(t_depth), _ptr(label), P, int(num_classes), weights,
                                    _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["sil"]), _ptr(out["sem"]),
                                    _ptr(scratch), stream), "sgr_mapping_loss_grad")
    return out


class FusedAdam:
    """Adam over a list of (param, grad, lo, hi) float32 tensors in one launch
    per step (sgr_adam_step), with the clamp applied after each update."""

    def __init__(self, groups, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        if len(groups) > L.SGR_MAX_ADAM_SEGMENTS:
            raise ValueError("too many parameter tensors for one fused Adam launch")
        self.groups = groups
        self.lr, self.b1, self.b2, self.eps = lr, betas[0], betas[1], eps
        self.m = [torch.zeros_like(p) for p, _, _, _ in groups]
        self.v = [torch.zeros_like(p) for p, _, _, _ in groups]
        self.t = 0
        self.segs = (L.sgr_adam_segment * len(groups))()
        for i, ((p, g, lo, hi), m, v) in enumerate(zip(groups, self.m, self.v)):
            self.segs[i] = L.sgr_adam_segment(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), float(lo), float(hi))

    def step(self):
        self.t += 1
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.m[0].device).cuda_stream)
        L.check(L.sgr_adam_step(self.segs, len(self.groups), self.lr, self.b1, self.b2, self.eps, self.t, stream),
                "sgr_adam_step")


def topk_select(dist: torch.Tensor, k: int, pixel: torch.Tensor | None = None, renormalize: bool = False):
    """Top-k (class, probability) of each row of dist [rows, C] (or of rows
    pixel[i]): new Gaussians' sparse semantics.  Returns (sem_idx uint8
    [n, k], sem_val float32 [n, k])."""
    dist = dist.to(torch.float32).contiguous()
    C = int(dist.shape[-1])
    dist2 = dist.reshape(-1, C)
    if pixel is not None:
        pixel = pixel.to(device=dist.device, dtype=torch.int64).contiguous()
    n = int(pixel.numel()) if pixel is not None else int(dist2.shape[0])
    idx = torch.empty((n, k), dtype=torch.uint8, device=dist.device)
    val = torch.empty((n, k), dtype=torch.float32, device=dist.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dist.device).cuda_stream)
    L.check(L.sgr_topk_select(_ptr(dist2), _ptr(pixel), n, C, int(k), int(bool(renormalize)), _ptr(idx), _ptr(val),
                              stream), "sgr_topk_select")
    return idx, val


def topk_update(dist: torch.Tensor, sem_idx: torch.Tensor, sem_val: torch.Tensor, rate: float,
                pixel: torch.Tensor | None = None):
    """In place: sem_val <- (1 - rate) sem_val + rate * dist[row][sem_idx]."""
    dist = dist.to(torch.float32).contiguous()
    C = int(dist.shape[-1])
    if pixel is not None:
        pixel = pixel.to(device=dist.device, dtype=torch.int64).contiguous()
    n, k = int(sem_idx.shape[0]), int(sem_idx.shape[1])
    stream = ctypes.c_void_p(torch.cuda.current_stream(dist.device).cuda_stream)
    L.check(L.sgr_topk_update(_ptr(dist.reshape(-1, C)), _ptr(pixel), n, C, k, _ptr(sem_idx.contiguous()),
                              float(rate), _ptr(sem_val), stream), "sgr_topk_update")
    return sem_val
