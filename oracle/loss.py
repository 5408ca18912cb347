"""FP64 oracle of the per-keyframe mapping loss and its gradient with respect
to the rendered maps.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU baseline leg
use this module; the product package never does.

Per view, with P pixels and per-pixel rendered colour C, depth D,
silhouette S and class distribution q (Eq. 1 and Eq. 3, Sec. 3.1):

    L = (1/P) sum_p [ m (w_d |D - D*| + w_c sum_ch |C - C*|) + w_s |S - 1| + w_sem L_sem ],
    m = [S > s_thr]   (held fixed: not differentiated)

The masked depth + 0.5 colour L1 follows Sec. 3.1's tracking/mapping loss;
the silhouette term pulls S to 1.  Two semantic terms are provided:

* cross-entropy against a label:  L_sem = -ln max(q_label, floor);
* the paper's semantic loss (Sec. 3.1, "Semantic Loss") against a dense
  pseudo-ground-truth distribution g:
      L_sem = M_H (lambda_HD D_HD(g, q) + lambda_cos (1 - cos(g, q))),
      M_H   = [H(g) < tau],  H(g) = -sum_m g_m ln g_m,  tau = ln k,
      D_HD  = (1/sqrt 2) sqrt( sum_m (sqrt(g_m + e) - sqrt(q_m + e))^2 ),
      cos   = <g, q> / (|g| |q|).

Readings where the paper is silent: the Hellinger distance is the standard
one with the 1/sqrt(2) factor; e = 1e-8 inside its square roots keeps the
slope finite where q_m = 0; a pixel with |q| = 0 or |g| = 0 has no cosine
(and gets no semantic term); every term is averaged over all P pixels.

Everything here is plain numpy in float64, written from the formulas above.
`flags` marks pixels where the FP32 kernel may legitimately take the other
side of a kink (a sign, the mask threshold, the cross-entropy floor or the
entropy threshold) than this FP64 reference.
"""
from __future__ import annotations

import numpy as np

DEFAULTS = dict(w_depth=1.0, w_rgb=0.5, w_sil=1.0, w_sem=1.0, sil_thresh=0.99, ce_floor=1e-6, lambda_hd=0.8,
                lambda_cos=0.2, tau=None, sqrt_eps=1e-8)


def entropy(g: np.ndarray) -> np.ndarray:
    """H(g) = -sum_m g_m ln g_m over the last axis, with 0 ln 0 = 0."""
    g = np.asarray(g, np.float64)
    t = np.where(g > 0, g * np.log(np.where(g > 0, g, 1.0)), 0.0)
    return -t.sum(-1)


def hellinger(g: np.ndarray, q: np.ndarray, e: float) -> np.ndarray:
    d = np.sqrt(g + e) - np.sqrt(q + e)
    return np.sqrt((d * d).sum(-1)) / np.sqrt(2.0)


def semantic_term(g: np.ndarray, q: np.ndarray, k: int, lambda_hd=0.8, lambda_cos=0.2, tau=None, sqrt_eps=1e-8):
    """Per-pixel M_H (lambda_HD D_HD + lambda_cos (1 - cos)) and its gradient
    with respect to q.  g, q: [..., C] float64.  Returns (value, grad, mask,
    entropy of g)."""
    with np.errstate(divide="ignore", invalid="ignore"):  # unselected branches of np.where
        return _semantic_term(np.asarray(g, np.float64), np.asarray(q, np.float64), k, lambda_hd, lambda_cos, tau,
                              sqrt_eps)


def _semantic_term(g, q, k, lambda_hd, lambda_cos, tau, sqrt_eps):
    tau = np.log(k) if tau is None or tau <= 0 else tau
    H = entropy(g)
    ng = np.sqrt((g * g).sum(-1))
    nq = np.sqrt((q * q).sum(-1))
    mask = (H < tau) & (ng > 0) & (nq > 0)
    e = sqrt_eps
    d = np.sqrt(g + e) - np.sqrt(q + e)
    root = np.sqrt((d * d).sum(-1))
    dhd = root / np.sqrt(2.0)
    safe_nq = np.where(nq > 0, nq, 1.0)
    safe_ng = np.where(ng > 0, ng, 1.0)
    cos = (g * q).sum(-1) / (safe_ng * safe_nq)
    value = np.where(mask, lambda_hd * dhd + lambda_cos * (1.0 - cos), 0.0)
    # d D_HD / d q_m = (1/sqrt 2) (1 / (2 root)) 2 d_m (-1 / (2 sqrt(q_m + e)))
    safe_root = np.where(root > 0, root, 1.0)
    g_hd = np.where(root[..., None] > 0, -d / (2.0 * np.sqrt(2.0) * safe_root[..., None] * np.sqrt(q + e)), 0.0)
    # d (1 - cos) / d q_m = -(g_m / (|g||q|) - cos q_m / |q|^2)
    g_cos = -(g / (safe_ng * safe_nq)[..., None] - cos[..., None] * q / (safe_nq * safe_nq)[..., None])
    grad = np.where(mask[..., None], lambda_hd * g_hd + lambda_cos * g_cos, 0.0)
    return value, grad, mask, H


def mapping_loss(maps: dict, targets: dict, num_classes: int, k: int, **kw):
    """Loss and dL/d(map) for one view.

    maps: rgb [H,W,3], depth [H,W], sil [H,W], sem [H,W,C] (the rendered
    maps, any float dtype; upcast to float64).  targets: rgb, depth and
    either `label` [H,W] (cross-entropy) or `sem` [H,W,C] (Hellinger +
    cosine with the entropy mask), or neither (no semantic term).
    Returns (loss, grads, flags) with grads in the layout of maps."""
    o = dict(DEFAULTS)
    o.update(kw)
    f = lambda a: np.asarray(a, np.float64)
    C_, D, S, Q = f(maps["rgb"]), f(maps["depth"]), f(maps["sil"]), f(maps["sem"])
    tc, td = f(targets["rgb"]), f(targets["depth"])
    P = D.size
    m = (S > o["sil_thresh"]).astype(np.float64)
    rd, rc = D - td, C_ - tc
    loss_px = m * (o["w_depth"] * np.abs(rd) + o["w_rgb"] * np.abs(rc).sum(-1)) + o["w_sil"] * np.abs(S - 1.0)
    g_depth = m * o["w_depth"] * np.sign(rd) / P
    g_rgb = m[..., None] * o["w_rgb"] * np.sign(rc) / P
    g_sil = o["w_sil"] * np.sign(S - 1.0) / P
    g_sem = np.zeros_like(Q)
    flags = (np.abs(S - o["sil_thresh"]) < 1e-5) | ((m > 0) & (np.abs(rd) < 1e-5 * (1.0 + np.abs(td))))
    flags |= (m > 0) & (np.abs(rc) < 1e-5).any(-1)
    if targets.get("sem") is not None:
        val, grad, mask, H = semantic_term(f(targets["sem"]), Q, k, o["lambda_hd"], o["lambda_cos"], o["tau"],
                                           o["sqrt_eps"])
        loss_px = loss_px + o["w_sem"] * val
        g_sem = o["w_sem"] * grad / P
        tau = np.log(k) if o["tau"] is None or o["tau"] <= 0 else o["tau"]
        flags |= np.abs(H - tau) < 1e-5
    elif targets.get("label") is not None:
        lab = np.asarray(targets["label"]).astype(np.int64)
        ql = np.take_along_axis(Q, lab[..., None], -1)[..., 0]
        fl = o["ce_floor"]
        loss_px = loss_px - o["w_sem"] * np.log(np.maximum(ql, fl))
        gl = np.where(ql > fl, -o["w_sem"] / np.where(ql > fl, ql, 1.0), 0.0) / P
        np.put_along_axis(g_sem, lab[..., None], gl[..., None], -1)
        flags |= np.abs(ql - fl) < 1e-5 * fl
    return float(loss_px.sum() / P), {"rgb": g_rgb, "depth": g_depth, "sil": g_sil, "sem": g_sem}, flags
