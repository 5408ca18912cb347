"""Python front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg import this module; the product package never does.

All inputs are upcast to float64 here; the C code then works in double
precision throughout.  Functions follow the paper's Sec. 3.1 (Eq. 1, Eq. 3)
and Sec. 3.2 (Eq. 4-6); see oracle.c for the per-function citations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB names another build of oracle.c (the sanitizer job of the CPU
# tests loads an ASan/UBSan build this way); it is used as built.
_LIB_ENV = os.environ.get("ORACLE_LIB")
_LIB = _LIB_ENV or os.path.join(_HERE, "liboracle.so")

# Default renderer constants (readings of the paper; see the design notes).
ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))
Z_NEAR = float(np.float32(0.2))
LOWPASS = float(np.float32(0.3))


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, -O2, OpenMP)."""
    if _LIB_ENV:
        return _LIB
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB_ENV and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.oracle_project.argtypes = [i64] + [P] * 6 + [P] * 7
        L.oracle_render.argtypes = [i64] + [P] * 7 + [i32, i32] + [P] * 3 + [i32, i32, P, i32, P] + [P] * 8
        L.oracle_render_branches.argtypes = ([i64] + [P] * 7 + [i32, i32] + [P] * 3 + [i32, i32, P, i64, P, i32]
                                             + [P] * 7)
        L.oracle_render_backward.argtypes = ([i64] + [P] * 7 + [i32, i32] + [P] * 3 + [i32, i32, P, P]
                                             + [P] * 4 + [P] * 6)
        L.oracle_project_backward.argtypes = [i64] + [P] * 5 + [P] * 4 + [P] * 3
        L.oracle_score.argtypes = [i32, i32, i32, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def camera_array(cam) -> np.ndarray:
    R = np.asarray(cam.R, dtype=np.float32).astype(np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float32).astype(np.float64).reshape(3)
    f = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    return np.concatenate([R, t, f, [cam.width, cam.height]]).astype(np.float64)


def config_array(alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, t_min=T_MIN, z_near=Z_NEAR, lowpass=LOWPASS,
                 tile_w=16, tile_h=16, sem_grad_to_geometry=0, margin_alpha=1e-5, margin_t=1e-4) -> np.ndarray:
    return np.array([alpha_min, alpha_max, t_min, z_near, lowpass, tile_w, tile_h, sem_grad_to_geometry,
                     margin_alpha, margin_t], dtype=np.float64)


def project(means, scales, quats, opacity, cam, cfg) -> dict:
    """Per-Gaussian projection into one camera (oracle.c oracle_project)."""
    means, scales, quats, opacity = _f64(means), _f64(scales), _f64(quats), _f64(opacity)
    n = means.shape[0]
    out = {
        "mean2d": np.zeros((n, 2)), "conic": np.zeros((n, 3)), "cov2d": np.zeros((n, 3)),
        "pcam": np.zeros((n, 3)), "rect": np.zeros((n, 4), np.int32), "zbits": np.zeros(n, np.uint32),
        "visible": np.zeros(n, np.int32),
    }
    ca = camera_array(cam)
    lib().oracle_project(n, _p(means), _p(scales), _p(quats), _p(opacity), _p(ca), _p(cfg),
                         _p(out["mean2d"]), _p(out["conic"]), _p(out["cov2d"]), _p(out["pcam"]),
                         _p(out["rect"]), _p(out["zbits"]), _p(out["visible"]))
    out["depth"] = out["pcam"][:, 2].copy()
    return out


def tile_grid(cam, tile_w=16, tile_h=16):
    return (cam.width + tile_w - 1) // tile_w, (cam.height + tile_h - 1) // tile_h


def reference_keys(projs, cams, tile_w=16, tile_h=16):
    """Reference key list over all views: one entry per (view, touched tile,
    visible Gaussian), sorted lexicographically by (view, tile id, fp32 depth
    bits, Gaussian id), plus [start, end) per global tile.  Tile id =
    ty * tiles_x + tx; global tile = per-view offset + tile id."""
    rows = []
    tile_off = [0]
    for v, (pr, cam) in enumerate(zip(projs, cams)):
        tx_n, ty_n = tile_grid(cam, tile_w, tile_h)
        ids = np.nonzero(pr["visible"])[0]
        r = pr["rect"][ids]
        tx0, tx1 = r[:, 0] // tile_w, r[:, 1] // tile_w
        ty0, ty1 = r[:, 2] // tile_h, r[:, 3] // tile_h
        cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
        rep = np.repeat(np.arange(len(ids)), cnt)
        local = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        wdt = (tx1 - tx0 + 1)[rep]
        tx = tx0[rep] + local % wdt
        ty = ty0[rep] + local // wdt
        tile = (ty * tx_n + tx).astype(np.int64)
        gid = ids[rep].astype(np.int64)
        rows.append(np.stack([np.full_like(tile, v), tile, pr["zbits"][gid].astype(np.int64), gid], 1))
        tile_off.append(tile_off[-1] + tx_n * ty_n)
    keys = np.concatenate(rows, 0) if rows else np.zeros((0, 4), np.int64)
    order = np.lexsort((keys[:, 3], keys[:, 2], keys[:, 1], keys[:, 0]))
    keys = keys[order]
    gt = np.asarray(tile_off[:-1], np.int64)[keys[:, 0]] + keys[:, 1]
    total = tile_off[-1]
    ranges = np.zeros((total, 2), np.int64)
    if len(gt):
        starts = np.searchsorted(gt, np.arange(total), side="left")
        ends = np.searchsorted(gt, np.arange(total), side="right")
        ranges[:, 0], ranges[:, 1] = starts, ends
        ranges[starts == ends] = 0
    return keys, ranges, np.asarray(tile_off, np.int64)


def _branch_arg(branch, H, W):
    if branch is None:
        return None
    b = np.ascontiguousarray(branch, dtype=np.uint32).reshape(H, W)
    return b


def render(proj, opacity, rgb, sem_val, sem_idx, num_classes, cam, cfg, brute=False, branch=None) -> dict:
    """Per-pixel compositing of Eq. 1 / Eq. 3 (oracle.c oracle_render).
    branch: optional [H, W] words choosing the outcomes of each pixel's
    flagged decisions (walk_pixel in oracle.c); None is the plain definition."""
    n = proj["mean2d"].shape[0]
    k = int(sem_val.shape[1])
    W, H, C = cam.width, cam.height, int(num_classes)
    opacity, rgb, sem_val = _f64(opacity), _f64(rgb), _f64(sem_val)
    sem_idx = np.ascontiguousarray(sem_idx, dtype=np.int32)
    out = {
        "rgb": np.zeros((H, W, 3)), "depth": np.zeros((H, W)), "sil": np.zeros((H, W)),
        "sem": np.zeros((H, W, C)), "t_final": np.zeros((H, W)), "n_contrib": np.zeros((H, W), np.int32),
        "flags": np.zeros((H, W), np.int32), "sig": np.zeros((H, W), np.uint64),
    }
    br = _branch_arg(branch, H, W)
    lib().oracle_render(n, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["depth"]), _p(opacity), _p(rgb),
                        _p(sem_val), _p(sem_idx), k, C, _p(proj["rect"]), _p(proj["zbits"]), _p(proj["visible"]),
                        W, H, _p(cfg), int(bool(brute)), _p(br), _p(out["rgb"]), _p(out["depth"]), _p(out["sil"]),
                        _p(out["sem"]), _p(out["t_final"]), _p(out["n_contrib"]), _p(out["flags"]), _p(out["sig"]))
    return out


def render_branches(proj, opacity, rgb, sem_val, sem_idx, num_classes, cam, cfg, pixels, nbits=4) -> dict:
    """Every outcome of the flagged decisions of the listed pixels
    (oracle.c oracle_render_branches).  pixels: [q, 2] (x, y).  Returns maps
    of shape [q, 2^nbits, ...] indexed by branch word, and "nflag" [q, 2^nbits],
    the flagged decisions each walk met (a walk that met more than nbits of
    them has outcomes left out)."""
    n = proj["mean2d"].shape[0]
    k = int(sem_val.shape[1])
    W, H, C = cam.width, cam.height, int(num_classes)
    opacity, rgb, sem_val = _f64(opacity), _f64(rgb), _f64(sem_val)
    sem_idx = np.ascontiguousarray(sem_idx, dtype=np.int32)
    pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32).reshape(-1, 2))
    q, nb = pix.shape[0], 1 << int(nbits)
    out = {"rgb": np.zeros((q, nb, 3)), "depth": np.zeros((q, nb)), "sil": np.zeros((q, nb)),
           "sem": np.zeros((q, nb, C)), "t_final": np.zeros((q, nb)), "n_contrib": np.zeros((q, nb), np.int32),
           "nflag": np.zeros((q, nb), np.int32)}
    if q == 0:
        return out
    rc = lib().oracle_render_branches(n, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["depth"]), _p(opacity),
                                      _p(rgb), _p(sem_val), _p(sem_idx), k, C, _p(proj["rect"]), _p(proj["zbits"]),
                                      _p(proj["visible"]), W, H, _p(cfg), q, _p(pix), int(nbits), _p(out["rgb"]),
                                      _p(out["depth"]), _p(out["sil"]), _p(out["sem"]), _p(out["t_final"]),
                                      _p(out["n_contrib"]), _p(out["nflag"]))
    if rc != 0:
        raise ValueError("nbits must lie in [0, 16]")
    return out


def render_backward(proj, opacity, rgb, sem_val, sem_idx, num_classes, cam, cfg, grads, branch=None) -> dict:
    """Analytic gradient with respect to the 2D parameters
    (oracle.c oracle_render_backward); `grads` holds dL/d{rgb,depth,sil,sem};
    `branch` as in render()."""
    n = proj["mean2d"].shape[0]
    k = int(sem_val.shape[1])
    W, H, C = cam.width, cam.height, int(num_classes)
    opacity, rgb, sem_val = _f64(opacity), _f64(rgb), _f64(sem_val)
    sem_idx = np.ascontiguousarray(sem_idx, dtype=np.int32)
    g = {key: _f64(grads[key]) for key in ("rgb", "depth", "sil", "sem")}
    out = {"mean2d": np.zeros((n, 2)), "conic": np.zeros((n, 3)), "opacity": np.zeros(n),
           "rgb": np.zeros((n, 3)), "depth": np.zeros(n), "sem_val": np.zeros((n, k))}
    lib().oracle_render_backward(n, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["depth"]), _p(opacity),
                                 _p(rgb), _p(sem_val), _p(sem_idx), k, C, _p(proj["rect"]), _p(proj["zbits"]),
                                 _p(proj["visible"]), W, H, _p(cfg), _p(_branch_arg(branch, H, W)), _p(g["rgb"]),
                                 _p(g["depth"]), _p(g["sil"]),
                                 _p(g["sem"]), _p(out["mean2d"]), _p(out["conic"]), _p(out["opacity"]),
                                 _p(out["rgb"]), _p(out["depth"]), _p(out["sem_val"]))
    return out


def project_backward(means, scales, quats, cam, proj, g2d) -> dict:
    """Chain rule from 2D to 3D parameters (oracle.c oracle_project_backward)."""
    means, scales, quats = _f64(means), _f64(scales), _f64(quats)
    n = means.shape[0]
    out = {"means": np.zeros((n, 3)), "scales": np.zeros((n, 3)), "quats": np.zeros((n, 4))}
    ca = camera_array(cam)
    lib().oracle_project_backward(n, _p(means), _p(scales), _p(quats), _p(ca), _p(proj["visible"]),
                                  _p(proj["conic"]), _p(_f64(g2d["mean2d"])), _p(_f64(g2d["conic"])),
                                  _p(_f64(g2d["depth"])), _p(out["means"]), _p(out["scales"]), _p(out["quats"]))
    return out


def score(maps, num_classes) -> dict:
    """Per-view n_empty and summed clipped entropy (oracle.c oracle_score)."""
    H, W = maps["n_contrib"].shape
    sem = _f64(maps["sem"])
    nc = np.ascontiguousarray(maps["n_contrib"], dtype=np.int32)
    ne = np.zeros(1, np.int64)
    hs = np.zeros(1, np.float64)
    h = np.zeros((H, W), np.float64)
    lib().oracle_score(W, H, int(num_classes), _p(sem), _p(nc), _p(ne), _p(hs), _p(h))
    return {"n_empty": int(ne[0]), "entropy_sum": float(hs[0]), "h": h}


# ---------------------------------------------------------------- helpers

def forward(scene_arrays, cam, cfg, num_classes, brute=False, branch=None):
    """Project + render one view.  scene_arrays: (means, scales, quats,
    opacity, rgb, sem_val, sem_idx)."""
    means, scales, quats, opacity, rgb, sem_val, sem_idx = scene_arrays
    pr = project(means, scales, quats, opacity, cam, cfg)
    mp = render(pr, opacity, rgb, sem_val, sem_idx, num_classes, cam, cfg, brute=brute, branch=branch)
    return pr, mp


def backward(scene_arrays, cam, cfg, num_classes, grads, proj=None, branch=None):
    """Full analytic gradient of sum_p <grads, maps> for one view, with
    respect to means, scales, quats, opacity, rgb, sem_val (`branch` as in
    render())."""
    means, scales, quats, opacity, rgb, sem_val, sem_idx = scene_arrays
    pr = proj if proj is not None else project(means, scales, quats, opacity, cam, cfg)
    g2 = render_backward(pr, opacity, rgb, sem_val, sem_idx, num_classes, cam, cfg, grads, branch=branch)
    g3 = project_backward(means, scales, quats, cam, pr, g2)
    return {"means": g3["means"], "scales": g3["scales"], "quats": g3["quats"], "opacity": g2["opacity"],
            "rgb": g2["rgb"], "sem_val": g2["sem_val"]}, g2


def loss_of_maps(maps, grads) -> float:
    return float(sum(np.sum(maps[key] * grads[key]) for key in ("rgb", "depth", "sil", "sem")))


def scene_arrays(scene):
    return (scene.means, scene.scales, scene.quats, scene.opacity, scene.rgb, scene.sem_val, scene.sem_idx)


def finite_difference(scene_arrays, cam, cfg, num_classes, grads, params=("means", "scales", "quats", "opacity",
                                                                             "rgb", "sem_val"), h_rel=1e-6):
    """Central finite differences in FP64 of L = sum_p <grads, maps> with
    respect to each coordinate of the named parameters.  Coordinates whose
    +h and -h renders take different per-pixel decisions (skip / blend /
    clamped blend / stop, hashed into the oracle's signature) are reported
    as NaN: the loss is not differentiable across such a decision."""
    names = ("means", "scales", "quats", "opacity", "rgb", "sem_val", "sem_idx")
    arrs = {nm: (np.array(a, dtype=np.float64) if nm != "sem_idx" else np.asarray(a))
            for nm, a in zip(names, scene_arrays)}
    out = {}
    for nm in params:
        base = arrs[nm]
        g = np.zeros(base.shape)
        flat = base.reshape(-1)
        gf = g.reshape(-1)
        for j in range(flat.size):
            x0 = flat[j]
            h = h_rel * max(1.0, abs(x0))
            vals, sigs = [], []
            for sgn in (1.0, -1.0):
                flat[j] = x0 + sgn * h
                _, mp = forward(tuple(arrs[n_] for n_ in names), cam, cfg, num_classes)
                vals.append(loss_of_maps(mp, grads))
                sigs.append(mp["sig"])
            flat[j] = x0
            gf[j] = (vals[0] - vals[1]) / (2 * h) if np.array_equal(sigs[0], sigs[1]) else np.nan
        out[nm] = g
    return out
