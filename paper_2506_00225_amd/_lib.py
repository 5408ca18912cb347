"""ctypes binding of libsgr.so (include/sgr.h), argument marshalling only.

Every function here has the name and argument order of the C entry point it
wraps.  There is no fallback: if the library is missing or does not load,
`lib()` raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# SGR_LIB names another build of the same library (the sanitizer job of the
# CPU tests loads a host-sanitized build this way).
LIB_PATH = os.environ.get("SGR_LIB") or os.path.join(_PKG, "libsgr.so")

c_float_p = ctypes.POINTER(ctypes.c_float)
P = ctypes.c_void_p

SGR_OK, SGR_EINVAL, SGR_ECAPACITY, SGR_EHIP, SGR_EUNSUPPORTED = 0, 1, 2, 3, 4


class sgr_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class sgr_config(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("z_near", ctypes.c_float), ("lowpass", ctypes.c_float), ("num_classes", ctypes.c_int32),
                ("top_k", ctypes.c_int32), ("sem_grad_to_geometry", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("sem_accumulators", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("score_workgroups", ctypes.c_int32), ("sem_passes", ctypes.c_int32), ("bwd_batch", ctypes.c_int32),
                ("radix_bits", ctypes.c_int32)]


SGR_ACC_AUTO, SGR_ACC_LDS, SGR_ACC_REGISTERS = 0, 1, 2
SGR_TILES_AUTO, SGR_TILES_XCD, SGR_TILES_LINEAR = 0, 1, 2


class sgr_gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", P), ("scales", P), ("quats", P), ("opacity", P), ("rgb", P),
                ("sem_val", P), ("sem_idx", P)]


class sgr_maps(ctypes.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("sil", P), ("sem", P), ("t_final", P), ("n_contrib", P)]


class sgr_map_grads(ctypes.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("sil", P), ("sem", P), ("sem_label", P), ("sem_at_label", P)]


class sgr_grads(ctypes.Structure):
    _fields_ = [("means", P), ("scales", P), ("quats", P), ("opacity", P), ("rgb", P), ("sem_val", P)]


class sgr_loss_view(ctypes.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("label", P), ("sem", P), ("g_rgb", P), ("g_depth", P), ("g_sil", P),
                ("g_sem", P), ("g_sem_at_label", P)]


class sgr_loss_config(ctypes.Structure):
    _fields_ = [(name, ctypes.c_float) for name in ("w_depth", "w_rgb", "w_sil", "w_sem", "sil_thresh", "ce_floor",
                                                     "lambda_hd", "lambda_cos", "entropy_tau", "sqrt_eps")]


class sgr_adam_segment(ctypes.Structure):
    _fields_ = [("p", P), ("g", P), ("m", P), ("v", P), ("n", ctypes.c_int64), ("lo", ctypes.c_float),
                ("hi", ctypes.c_float)]


SGR_MAX_ADAM_SEGMENTS = 8


class sgr_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("voxel", ctypes.c_float),
                ("origin", ctypes.c_float * 3)]


class sgr_sampling(ctypes.Structure):
    _fields_ = [("step", ctypes.c_float), ("directions", ctypes.c_int32), ("z_min", ctypes.c_float),
                ("z_max", ctypes.c_float)]


class sgr_layout(ctypes.Structure):
    _fields_ = [(name, ctypes.c_size_t) for name in (
        "total_bytes", "counters", "views", "proj_count", "proj_zbits", "pair_rec", "pair_lin", "order",
        "sorted_keys", "sorted_vals", "key_owner", "ranges", "tile_offsets")] + [
        ("num_tiles", ctypes.c_int64), ("num_pixels", ctypes.c_int64), ("vn", ctypes.c_int64)]


EXPORTS = (
    "sgr_workspace_size", "sgr_workspace_layout", "sgr_project", "sgr_bin", "sgr_render_forward",
    "sgr_render_forward_loss", "sgr_render_forward_dense",
    "sgr_render_backward", "sgr_render_backward_tiles", "sgr_render_backward_gather", "sgr_score_views", "sgr_score_maps_workspace_size", "sgr_score_maps",
    "sgr_read_status", "sgr_status_string", "sgr_mapping_loss_grad", "sgr_adam_step",
    "sgr_candidates_workspace_size", "sgr_generate_candidates", "sgr_score_poses", "sgr_combine_scores",
    "sgr_topk_select", "sgr_topk_update", "sgr_score_maps_noalloc", "sgr_render_backward_gather_adam",
)

_lib = None


def lib():
    """Loads libsgr.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsgr.so not found at {LIB_PATH}: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    cam_p, cfg_p = ctypes.POINTER(sgr_camera), ctypes.POINTER(sgr_config)
    g_p = ctypes.POINTER(sgr_gaussians)
    L.sgr_workspace_size.argtypes = [i64, cam_p, i32, cfg_p, i64]
    L.sgr_workspace_size.restype = sz
    L.sgr_workspace_layout.argtypes = [i64, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_layout)]
    L.sgr_workspace_layout.restype = i32
    L.sgr_project.argtypes = [g_p, cam_p, i32, cfg_p, i64, P, sz, P]
    L.sgr_project.restype = i32
    L.sgr_bin.argtypes = [g_p, cam_p, i32, cfg_p, i64, P, P, sz, P]
    L.sgr_bin.restype = i32
    L.sgr_render_forward.argtypes = [g_p, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_maps), P, sz, P]
    L.sgr_render_forward.restype = i32
    L.sgr_render_forward_loss.argtypes = [g_p, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_maps),
                                          ctypes.POINTER(sgr_loss_view), ctypes.POINTER(sgr_loss_config), P, P, sz, P]
    L.sgr_render_forward_loss.restype = i32
    L.sgr_render_forward_dense.argtypes = [g_p, P, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_maps), P, sz, P]
    L.sgr_render_forward_dense.restype = i32
    L.sgr_render_backward.argtypes = [g_p, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_map_grads),
                                      ctypes.POINTER(sgr_grads), P, sz, P]
    L.sgr_render_backward.restype = i32
    L.sgr_render_backward_tiles.argtypes = [g_p, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_map_grads), P, sz, P]
    L.sgr_render_backward_tiles.restype = i32
    L.sgr_render_backward_gather.argtypes = [g_p, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_grads), P, sz, P]
    L.sgr_render_backward_gather.restype = i32
    L.sgr_score_views.argtypes = [g_p, cam_p, i32, cfg_p, i64, P, P, P, sz, P]
    L.sgr_score_views.restype = i32
    L.sgr_score_maps_workspace_size.argtypes = [i32, i32]
    L.sgr_score_maps_workspace_size.restype = sz
    L.sgr_score_maps.argtypes = [P, P, i32, i32, i32, P, P, P, sz, P]
    L.sgr_score_maps.restype = i32
    L.sgr_read_status.argtypes = [P, P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sgr_read_status.restype = i32
    L.sgr_mapping_loss_grad.argtypes = [P] * 7 + [i64, i32, P] + [P] * 5 + [P]
    L.sgr_mapping_loss_grad.restype = i32
    L.sgr_adam_step.argtypes = [ctypes.POINTER(sgr_adam_segment), i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, i32, P]
    L.sgr_adam_step.restype = i32
    grid_p, samp_p = ctypes.POINTER(sgr_grid), ctypes.POINTER(sgr_sampling)
    L.sgr_candidates_workspace_size.argtypes = [grid_p, samp_p]
    L.sgr_candidates_workspace_size.restype = sz
    L.sgr_generate_candidates.argtypes = [grid_p, P, P, samp_p, i64, P, P, P, P, sz, P]
    L.sgr_generate_candidates.restype = i32
    L.sgr_score_poses.argtypes = [g_p, cam_p, i32, P, cfg_p, i64, P, P, P, sz, P]
    L.sgr_score_poses.restype = i32
    L.sgr_combine_scores.argtypes = [i32, P, P, P, ctypes.POINTER(ctypes.c_float), i64, ctypes.c_float, P, P, P, P]
    L.sgr_combine_scores.restype = i32
    L.sgr_topk_select.argtypes = [P, P, i64, i32, i32, i32, P, P, P]
    L.sgr_topk_select.restype = i32
    L.sgr_topk_update.argtypes = [P, P, i64, i32, i32, P, ctypes.c_float, P, P]
    L.sgr_topk_update.restype = i32
    L.sgr_render_backward_gather_adam.argtypes = [g_p, cam_p, i32, cfg_p, i64, ctypes.POINTER(sgr_adam_segment),
                                                  ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, i32,
                                                  P, sz, P]
    L.sgr_render_backward_gather_adam.restype = i32
    L.sgr_score_maps_noalloc.argtypes = [P, P, i32, i32, i32, P, P, P]
    L.sgr_score_maps_noalloc.restype = i32
    L.sgr_status_string.argtypes = [i32]
    L.sgr_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


class SgrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        msg = lib().sgr_status_string(int(status)).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def check(status: int, where: str) -> None:
    if status != SGR_OK:
        raise SgrError(status, where)


# ---------------------------------------------------------------- same-name wrappers

def sgr_workspace_size(n, cams, num_views, cfg, key_capacity):
    return lib().sgr_workspace_size(n, cams, num_views, ctypes.byref(cfg), key_capacity)


def sgr_workspace_layout(n, cams, num_views, cfg, key_capacity):
    out = sgr_layout()
    check(lib().sgr_workspace_layout(n, cams, num_views, ctypes.byref(cfg), key_capacity, ctypes.byref(out)),
          "sgr_workspace_layout")
    return out


def sgr_project(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, stream):
    return lib().sgr_project(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, workspace,
                             workspace_bytes, stream)


def sgr_bin(g, cams, num_views, cfg, key_capacity, d_num_keys, workspace, workspace_bytes, stream):
    return lib().sgr_bin(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, d_num_keys, workspace,
                         workspace_bytes, stream)


def sgr_render_forward(g, cams, num_views, cfg, key_capacity, maps, workspace, workspace_bytes, stream):
    return lib().sgr_render_forward(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, maps,
                                    workspace, workspace_bytes, stream)


def sgr_render_forward_loss(g, cams, num_views, cfg, key_capacity, maps, views, loss_cfg, loss, workspace,
                            workspace_bytes, stream):
    return lib().sgr_render_forward_loss(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, maps,
                                         views, ctypes.byref(loss_cfg), loss, workspace, workspace_bytes, stream)


def sgr_render_forward_dense(g, dense_sem, cams, num_views, cfg, key_capacity, maps, workspace, workspace_bytes,
                             stream):
    return lib().sgr_render_forward_dense(ctypes.byref(g), dense_sem, cams, num_views, ctypes.byref(cfg),
                                          key_capacity, maps, workspace, workspace_bytes, stream)


def sgr_render_backward(g, cams, num_views, cfg, key_capacity, dl, grads, workspace, workspace_bytes, stream):
    return lib().sgr_render_backward(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, dl,
                                     ctypes.byref(grads), workspace, workspace_bytes, stream)


def sgr_render_backward_tiles(g, cams, num_views, cfg, key_capacity, dl, workspace, workspace_bytes, stream):
    return lib().sgr_render_backward_tiles(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, dl,
                                           workspace, workspace_bytes, stream)


def sgr_render_backward_gather(g, cams, num_views, cfg, key_capacity, grads, workspace, workspace_bytes, stream):
    return lib().sgr_render_backward_gather(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity,
                                            ctypes.byref(grads), workspace, workspace_bytes, stream)


def sgr_score_views(g, cams, num_views, cfg, key_capacity, n_empty, entropy_sum, workspace, workspace_bytes, stream):
    return lib().sgr_score_views(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity, n_empty,
                                 entropy_sum, workspace, workspace_bytes, stream)


def sgr_score_maps_workspace_size(width, height):
    return lib().sgr_score_maps_workspace_size(width, height)


def sgr_score_maps(sem, n_contrib, width, height, num_classes, n_empty, entropy_sum, workspace, workspace_bytes,
                   stream):
    return lib().sgr_score_maps(sem, n_contrib, width, height, num_classes, n_empty, entropy_sum, workspace,
                                workspace_bytes, stream)


# the static scratch of sgr_score_maps_noalloc (include/sgr.h) holds the
# partial sums of at most this many pixels
SGR_NOALLOC_MAX_PIXELS = 16 * 1024 * 1024


def sgr_score_maps_noalloc(sem, n_contrib, width, height, num_classes, n_empty, entropy_sum, stream):
    return lib().sgr_score_maps_noalloc(sem, n_contrib, width, height, num_classes, n_empty, entropy_sum, stream)


def sgr_render_backward_gather_adam(g, cams, num_views, cfg, key_capacity, segments, lr, beta1, beta2, eps, step,
                                    workspace, workspace_bytes, stream):
    return lib().sgr_render_backward_gather_adam(ctypes.byref(g), cams, num_views, ctypes.byref(cfg), key_capacity,
                                                 segments, lr, beta1, beta2, eps, step, workspace, workspace_bytes,
                                                 stream)


def sgr_read_status(workspace, stream):
    nv, nk = ctypes.c_int64(0), ctypes.c_int64(0)
    st = lib().sgr_read_status(workspace, stream, ctypes.byref(nv), ctypes.byref(nk))
    return st, nv.value, nk.value


def sgr_status_string(status):
    return lib().sgr_status_string(int(status)).decode()


def sgr_mapping_loss_grad(rgb, depth, sil, sem, t_rgb, t_depth, label, num_pixels, num_classes, weights, g_rgb,
                          g_depth, g_sil, g_sem, scratch, stream):
    w = (ctypes.c_float * 5)(*[float(x) for x in weights])
    return lib().sgr_mapping_loss_grad(rgb, depth, sil, sem, t_rgb, t_depth, label, num_pixels, num_classes, w, g_rgb,
                                       g_depth, g_sil, g_sem, scratch, stream)


def sgr_adam_step(segments, num_segments, lr, beta1, beta2, eps, step, stream):
    return lib().sgr_adam_step(segments, num_segments, lr, beta1, beta2, eps, step, stream)


def sgr_candidates_workspace_size(grid, sampling):
    return lib().sgr_candidates_workspace_size(ctypes.byref(grid), ctypes.byref(sampling))


def sgr_generate_candidates(grid, free_now, free_before, sampling, capacity, poses, positions, d_count, workspace,
                            workspace_bytes, stream):
    return lib().sgr_generate_candidates(ctypes.byref(grid), free_now, free_before, ctypes.byref(sampling), capacity,
                                         poses, positions, d_count, workspace, workspace_bytes, stream)


def sgr_score_poses(g, intrinsics, num_views, poses, cfg, key_capacity, n_empty, entropy_sum, workspace,
                    workspace_bytes, stream):
    return lib().sgr_score_poses(ctypes.byref(g), intrinsics, num_views, poses, ctypes.byref(cfg), key_capacity,
                                 n_empty, entropy_sum, workspace, workspace_bytes, stream)


def sgr_combine_scores(num_views, n_empty, entropy_sum, positions, current, pixels, prune_fraction, score, pruned, best,
                       stream):
    cur = (ctypes.c_float * 3)(*[float(x) for x in current])
    return lib().sgr_combine_scores(num_views, n_empty, entropy_sum, positions, cur, pixels, prune_fraction, score,
                                    pruned, best, stream)


def sgr_topk_select(dist, pixel, n, num_classes, k, renormalize, sem_idx, sem_val, stream):
    return lib().sgr_topk_select(dist, pixel, n, num_classes, k, renormalize, sem_idx, sem_val, stream)


def sgr_topk_update(dist, pixel, n, num_classes, k, sem_idx, rate, sem_val, stream):
    return lib().sgr_topk_update(dist, pixel, n, num_classes, k, sem_idx, rate, sem_val, stream)
