"""Helpers shared by the GPU parity tests (import only from tests)."""
import numpy as np
import torch

from oracle import oracle as O
from paper_2506_00225_amd import Frame, Gaussians, make_config

LN2 = 0.6931471805599453


def frame_for(sc, cams=None, cap=None, semgeo=0, lowpass=None, acc=0, passes=0):
    kw = {} if lowpass is None else {"lowpass": lowpass}
    cfg = make_config(sc.num_classes, sc.k, sem_grad_to_geometry=semgeo, sem_accumulators=acc, sem_passes=passes,
                      **kw)
    cams = sc.cameras if cams is None else cams
    return Frame(sc.n, cams, cfg, key_capacity=cap, device="cuda")


def oracle_cfg(semgeo=0, lowpass=None):
    return O.config_array(sem_grad_to_geometry=semgeo, **({} if lowpass is None else {"lowpass": float(np.float32(lowpass))}))


def ws_u32(fr, off, count):
    return fr.ws[off:off + 4 * count].view(torch.int32).cpu().numpy().view(np.uint32)


def ws_f32(fr, off, count):
    return fr.ws[off:off + 4 * count].view(torch.float32).cpu().numpy()


def counters(fr):
    return ws_u32(fr, 0, 16)


def gpu_keys(fr):
    """(view, tile, zbits, id) of every sorted key, and ranges per tile."""
    lay = fr.layout
    c = counters(fr)
    K = int(c[5])
    nvis = int(c[1])
    gt = ws_u32(fr, lay.sorted_keys, K).astype(np.int64)
    sgp = ws_u32(fr, lay.sorted_gauss, K).astype(np.int64)
    order = ws_u32(fr, lay.order, nvis).astype(np.int64)
    zb = ws_u32(fr, lay.proj_zbits, lay.vn).astype(np.int64)
    lin = order[sgp]
    view = lin // fr.n
    gid = lin % fr.n
    tile_off = np.cumsum([0] + [((c_.width + 15) // 16) * ((c_.height + 15) // 16) for c_ in fr.cam_list])
    tile = gt - tile_off[view]
    keys = np.stack([view, tile, zb[lin], gid], 1)
    rng = ws_u32(fr, lay.ranges, 2 * lay.num_tiles).reshape(-1, 2).astype(np.int64)
    return keys, rng


def gpu_proj(fr):
    """Projected records of view 0 (indexed by Gaussian id): visible, rect,
    zbits, tile count, mean2d, conic; taken from the front-to-back records."""
    lay = fr.layout
    n = fr.n
    cnt = ws_u32(fr, lay.proj_count, n)
    zb = ws_u32(fr, lay.proj_zbits, n)
    nvis = int(counters(fr)[1])
    order = ws_u32(fr, lay.order, nvis).astype(np.int64)
    srec = fr.ws[lay.sorted_rec:lay.sorted_rec + 48 * nvis].view(torch.float32).cpu().numpy().reshape(nvis, 12)
    rec = np.zeros((n, 12), np.float32)
    mask = order < n  # view 0 only
    rec[order[mask]] = srec[mask]
    ri = rec.view(np.int32)
    ru = rec.view(np.uint32)
    # the record holds 0.5 - fraction of the mean (fp32)
    mean2d = np.stack([ri[:, 0] + (0.5 - rec[:, 2].astype(np.float64)), ri[:, 1] + (0.5 - rec[:, 3].astype(np.float64))], 1)
    ca = rec[:, 4].astype(np.float64) * 2 * LN2
    cb = rec[:, 5].astype(np.float64) * ca
    cc = rec[:, 6].astype(np.float64) * 2 * LN2 + rec[:, 5].astype(np.float64) * cb
    rect = np.stack([ru[:, 8] & 0xffff, ru[:, 8] >> 16, ru[:, 9] & 0xffff, ru[:, 9] >> 16], 1).astype(np.int32)
    return {"visible": cnt > 0, "count": cnt, "zbits": zb, "mean2d": mean2d, "conic": np.stack([ca, cb, cc], 1),
            "rect": rect, "opacity": rec[:, 7]}


def tiles_touched(rect):
    return ((rect[:, 1] // 16 - rect[:, 0] // 16 + 1) * (rect[:, 3] // 16 - rect[:, 2] // 16 + 1)).astype(np.uint32)


def compare_maps(got: dict, want: dict, flags: np.ndarray, atol=1e-4):
    """Element-wise comparison on unflagged pixels; flagged pixels (a
    decision within the oracle's margin of a threshold, where both outcomes
    are correct) only have to satisfy the compositing invariants."""
    ok = flags == 0
    report = {"flagged": int((~ok).sum())}
    for key in ("rgb", "depth", "sil", "sem", "t_final"):
        if key not in got or got[key] is None:
            continue
        g = got[key].astype(np.float64).reshape(want[key].shape)
        err = np.abs(g - want[key])[ok]
        report[key] = float(err.max()) if err.size else 0.0
        assert report[key] <= atol, (key, report)
    nc = got["n_contrib"].reshape(want["n_contrib"].shape)
    assert np.array_equal(nc[ok], want["n_contrib"][ok]), report
    return report


def tainted_gaussians(proj, flags):
    """Gaussians whose pixel rectangle covers a flagged pixel."""
    ys, xs = np.nonzero(flags)
    bad = np.zeros(proj["rect"].shape[0], bool)
    r = proj["rect"]
    vis = proj["visible"] == 1
    for y, x in zip(ys, xs):
        bad |= vis & (r[:, 0] <= x) & (r[:, 1] >= x) & (r[:, 2] <= y) & (r[:, 3] >= y)
    return bad


def compare_grads(got: dict, want: dict, exclude: np.ndarray, rtol=1e-3):
    """Per parameter tensor: relative L2 error over all Gaussians <= rtol, and
    element-wise |d| <= rtol |ref| + rtol rms(ref) on Gaussians that cover no
    flagged pixel (where both compositing outcomes are correct)."""
    keep = ~exclude
    report = {"excluded": int(exclude.sum())}
    for name, ref in want.items():
        gall = got[name].astype(np.float64)
        dall = gall - ref
        nrm = float(np.linalg.norm(dall) / (np.linalg.norm(ref) + 1e-30))
        d, r = dall[keep], ref[keep]
        rms = float(np.sqrt(np.mean(ref * ref))) + 1e-30
        worst = float(np.max(np.abs(d) - rtol * np.abs(r) - rtol * rms)) if d.size else -1.0
        report[name] = (nrm, worst)
        assert nrm <= rtol, (name, report)
        assert worst <= 0, (name, report)
    return report


def to_np(t):
    return t.detach().cpu().numpy()
