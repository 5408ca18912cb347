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
    svals = ws_u32(fr, lay.sorted_vals, K).astype(np.int64)
    rec = ws_u32(fr, lay.key_owner, K).astype(np.int64)[svals]
    pair_lin = ws_u32(fr, lay.pair_lin, nvis).astype(np.int64)
    zb = ws_u32(fr, lay.proj_zbits, lay.vn).astype(np.int64)
    lin = pair_lin[rec]
    view = lin // fr.n
    gid = lin % fr.n
    tile_off = np.cumsum([0] + [((c_.width + 15) // 16) * ((c_.height + 15) // 16) for c_ in fr.cam_list])
    tile = gt - tile_off[view]
    keys = np.stack([view, tile, zb[lin], gid], 1)
    rng = ws_u32(fr, lay.ranges, 2 * lay.num_tiles).reshape(-1, 2).astype(np.int64)
    return keys, rng


def gpu_proj(fr):
    """Projected records of view 0 (indexed by Gaussian id): visible, rect,
    zbits, tile count, mean2d, conic; taken from the pairs' records."""
    lay = fr.layout
    n = fr.n
    cnt = ws_u32(fr, lay.proj_count, n)
    zb = ws_u32(fr, lay.proj_zbits, n)
    nvis = int(counters(fr)[1])
    pair_lin = ws_u32(fr, lay.pair_lin, nvis).astype(np.int64)
    prec = fr.ws[lay.pair_rec:lay.pair_rec + 48 * nvis].view(torch.float32).cpu().numpy().reshape(nvis, 12)
    rec = np.zeros((n, 12), np.float32)
    mask = pair_lin < n  # view 0 only
    rec[pair_lin[mask]] = prec[mask]
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


class OracleView:
    """The oracle's projection and maps of one view (the plain definition),
    and, once `resolve` has seen the GPU's maps, the outcome of every flagged
    decision the GPU took (a branch word per pixel): maps and gradients of
    the oracle on those branches are then compared with the GPU everywhere."""

    def __init__(self, arrays, cam, cfg, num_classes):
        self.arrays, self.cam, self.cfg, self.C = arrays, cam, cfg, int(num_classes)
        self.pr, self.mp = O.forward(arrays, cam, cfg, num_classes)
        H, W = cam.height, cam.width
        self.branch = np.zeros((H, W), np.uint32)
        self.unresolved = np.zeros((H, W), bool)

    @staticmethod
    def of_scene(sc, cam=None, cfg=None):
        return OracleView(O.scene_arrays(sc), sc.cameras[0] if cam is None else cam,
                          oracle_cfg() if cfg is None else cfg, sc.num_classes)

    @property
    def flags(self):
        return self.mp["flags"]

    def resolve(self, got: dict, atol=1e-4, nbits=4):
        """At each flagged pixel, the outcome of its flagged decisions whose
        maps the GPU's match (n_contrib exactly, every channel in `got`
        within atol; the closest if several).  A pixel none matches fails
        the comparison unless one of its walks met more flagged decisions
        than the nbits enumerated (then it is counted as unresolved)."""
        ys, xs = np.nonzero(self.flags)
        rep = {"flagged": int(len(ys)), "unresolved": 0, "non_default": 0}
        if not len(ys):
            return rep
        _, _, _, opacity, rgb, sem_val, sem_idx = self.arrays
        b = O.render_branches(self.pr, opacity, rgb, sem_val, sem_idx, self.C, self.cam, self.cfg,
                              np.stack([xs, ys], 1), nbits=nbits)
        q, nrow = len(ys), 1 << nbits
        err = np.zeros((q, nrow))
        for key in ("rgb", "depth", "sil", "sem", "t_final"):
            if got.get(key) is None:
                continue
            g = got[key].astype(np.float64).reshape(self.mp[key].shape)[ys, xs]
            d = np.abs(b[key] - g[:, None])
            err = np.maximum(err, d.reshape(q, nrow, -1).max(-1))
        nc = got["n_contrib"].reshape(self.mp["n_contrib"].shape)[ys, xs]
        match = (b["n_contrib"] == nc[:, None]) & (err <= atol)
        best = np.argmin(np.where(match, err, np.inf), axis=1)
        ok = match.any(1)
        beyond = b["nflag"].max(1) > nbits
        bad = ~ok & ~beyond
        assert not bad.any(), ("flagged pixels no branch explains", int(bad.sum()), list(zip(xs[bad], ys[bad]))[:5])
        self.branch[ys, xs] = np.where(ok, best, 0).astype(np.uint32)
        self.unresolved[ys[~ok], xs[~ok]] = True
        rep["unresolved"] = int((~ok).sum())
        rep["non_default"] = int((ok & (best != 0)).sum())
        return rep

    def maps(self):
        """The oracle's maps on the resolved branches."""
        _, _, _, opacity, rgb, sem_val, sem_idx = self.arrays
        return O.render(self.pr, opacity, rgb, sem_val, sem_idx, self.C, self.cam, self.cfg, branch=self.branch)

    def backward(self, grads):
        """The oracle's analytic gradient on the resolved branches."""
        want, _ = O.backward(self.arrays, self.cam, self.cfg, self.C, grads, proj=self.pr, branch=self.branch)
        return want

    def excluded(self):
        """Gaussians whose rectangle covers an unresolved pixel."""
        return tainted_gaussians(self.pr, self.unresolved)


def compare_maps(got: dict, want, flags=None, atol=1e-4):
    """Maps within atol and n_contrib exact.  With an OracleView, flagged
    pixels (a decision within the oracle's margin of a threshold, where
    either outcome is correct) are compared with the outcome the GPU took
    (OracleView.resolve), and also checked for S + T_final = 1; with plain
    oracle maps they only get that invariant."""
    view = want if isinstance(want, OracleView) else None
    if view is not None:
        rep = view.resolve(got, atol=atol)
        want, flags = view.maps(), view.unresolved
    ok = flags == 0
    report = {"flagged": int((~ok).sum())} if view is None else rep
    for key in ("rgb", "depth", "sil", "sem", "t_final"):
        if key not in got or got[key] is None:
            continue
        g = got[key].astype(np.float64).reshape(want[key].shape)
        err = np.abs(g - want[key])[ok]
        report[key] = float(err.max()) if err.size else 0.0
        assert report[key] <= atol, (key, report)
    nc = got["n_contrib"].reshape(want["n_contrib"].shape)
    assert np.array_equal(nc[ok], want["n_contrib"][ok]), report
    if got.get("sil") is not None and got.get("t_final") is not None:
        s = got["sil"].astype(np.float64).reshape(want["sil"].shape) + got["t_final"].reshape(want["sil"].shape)
        assert np.abs(s - 1).max() <= 2e-5, report
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


def compare_grads(got: dict, want: dict, exclude: np.ndarray, rtol=1e-3, visible=None, max_excluded=0.01):
    """Per parameter tensor: relative L2 error over all Gaussians <= rtol, and
    element-wise |d| <= rtol |ref| + rtol rms(ref) on every Gaussian but the
    excluded ones (those covering a flagged pixel whose outcome could not be
    resolved), which may be at most max_excluded of the visible ones."""
    keep = ~exclude
    report = {"excluded": int(exclude.sum())}
    if visible is not None:
        nvis = int(np.count_nonzero(visible))
        report["visible"] = nvis
        report["excluded_frac"] = report["excluded"] / max(nvis, 1)
        assert report["excluded_frac"] <= max_excluded, report
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
