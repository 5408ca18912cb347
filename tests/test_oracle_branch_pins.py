"""Pins of the oracle's flagged-decision branches (walk_pixel's `branch`
word) and of its pixel rectangle.

Where single and double precision may legitimately decide a threshold test
differently (alpha near alpha_min, T (1 - alpha) near t_min), the oracle
can take the other outcome of each such decision.  These tests fix what the
other outcome is, against things other than the oracle itself:

* closed forms: one isotropic Gaussian whose alpha at a pixel sits just
  below the cutoff, and flat layers whose transmittance sits just above or
  below the stop (Eq. 1 with the cutoff and stop rules);
* the plain definition with the threshold moved across the decision (a
  flipped decision is that definition, maps and gradients alike);
* invariants of every enumerated outcome.

The rectangle pins check tightness by a numerical search along pixel-centre
lines (no use of the closed-form extent), and the far-mean cull reading.
CPU only.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2506_00225_amd import scenes


def _scene(means, scales, quats, opacity, rgb, sem_val, sem_idx, C, cam):
    f = lambda a: np.asarray(a, dtype=np.float32)
    return scenes.Scene(f(means), f(scales), f(quats), f(opacity), f(rgb), f(sem_val),
                        np.asarray(sem_idx, dtype=np.uint8), C, [cam])


def _cam(w, h, f):
    return scenes.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, w / 2, h / 2, w, h)


def _arrays(sc):
    return O.scene_arrays(sc)


def _branches(sc, pixels, nbits=2, cfg=None):
    cfg = O.config_array() if cfg is None else cfg
    cam = sc.cameras[0]
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, cfg)
    return O.render_branches(pr, sc.opacity, sc.rgb, sc.sem_val, sc.sem_idx, sc.num_classes, cam, cfg, pixels,
                             nbits=nbits)


# ---------------------------------------------------------------- alpha cutoff

def _cutoff_scene(rel):
    """One isotropic Gaussian on the axis of a 32x32 view (f = 30, z = 2,
    s = 0.05) whose alpha at the centre of pixel (18, 16) (offset (2.5, 0.5)
    from the mean) is alpha_min (1 + rel)."""
    f, z, s = 30.0, 2.0, 0.05
    s32, z32 = float(np.float32(s)), float(np.float32(z))
    var = (f * s32 / z32) ** 2 + O.LOWPASS
    G = math.exp(-(2.5 ** 2 + 0.5 ** 2) / (2 * var))
    o = float(np.float32(O.ALPHA_MIN * (1 + rel) / G))
    cam = _cam(32, 32, f)
    sc = _scene([[0, 0, z]], [[s] * 3], [[1, 0, 0, 0]], [o], [[0.2, 0.5, 0.9]], [[0.7, 0.3]], [[1, 3]], 4, cam)
    return sc, o * G


def test_alpha_cutoff_flip_blends_the_skipped_gaussian():
    """alpha = alpha_min (1 - 3e-6): skipped by default (n = 0); the other
    outcome blends it, C = c alpha, D = z alpha, S = alpha, P_m = v_m alpha,
    T = 1 - alpha (Eq. 1 / Eq. 3 with one Gaussian)."""
    sc, alpha = _cutoff_scene(-3e-6)
    assert alpha < O.ALPHA_MIN and abs(alpha / O.ALPHA_MIN - 1) < 1e-5
    b = _branches(sc, [(18, 16)], nbits=1)
    assert list(b["nflag"][0]) == [1, 1]
    assert b["n_contrib"][0, 0] == 0 and b["t_final"][0, 0] == 1.0 and not b["sem"][0, 0].any()
    assert b["n_contrib"][0, 1] == 1
    c = np.float32([0.2, 0.5, 0.9]).astype(np.float64)
    v = np.float32([0.7, 0.3]).astype(np.float64)
    assert np.allclose(b["rgb"][0, 1], c * alpha, rtol=1e-12)
    assert math.isclose(b["depth"][0, 1], 2.0 * alpha, rel_tol=1e-12)
    assert math.isclose(b["sil"][0, 1], alpha, rel_tol=1e-12)
    assert math.isclose(b["t_final"][0, 1], 1 - alpha, rel_tol=1e-14)
    assert np.allclose(b["sem"][0, 1, [1, 3]], v * alpha, rtol=1e-12)


def test_alpha_cutoff_flip_skips_the_blended_gaussian():
    """alpha = alpha_min (1 + 3e-6): blended by default; the other outcome
    skips it and leaves the pixel empty."""
    sc, alpha = _cutoff_scene(3e-6)
    assert alpha >= O.ALPHA_MIN
    b = _branches(sc, [(18, 16)], nbits=1)
    assert b["n_contrib"][0, 0] == 1 and math.isclose(b["sil"][0, 0], alpha, rel_tol=1e-12)
    assert b["n_contrib"][0, 1] == 0 and b["sil"][0, 1] == 0 and b["t_final"][0, 1] == 1.0


def test_unflagged_pixel_has_one_outcome():
    """A pixel whose alpha is far from the cutoff meets no flagged decision:
    every branch word gives the plain result."""
    sc, _ = _cutoff_scene(-3e-6)
    b = _branches(sc, [(16, 16)], nbits=2)
    assert not b["nflag"].any()
    for key in ("rgb", "sil", "sem", "t_final", "n_contrib"):
        for j in range(1, 4):
            assert np.array_equal(b[key][0, j], b[key][0, 0]), key


# ---------------------------------------------------------------- transmittance stop

def _stop_scene(rel):
    """Flat layers (alpha = o to 1e-10 everywhere): three of o = 0.9, then a
    fourth whose T (1 - alpha) is t_min (1 + rel), then o = 0.5."""
    o3 = float(np.float32(0.9))
    T3 = (1 - o3) ** 3
    o4 = float(np.float32(1 - O.T_MIN * (1 + rel) / T3))
    ops = [o3, o3, o3, o4, 0.5]
    n = len(ops)
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [0, 1, 1]]
    cam = _cam(8, 8, 8.0)
    sc = _scene([[0, 0, 1.0 + 0.1 * i] for i in range(n)], [[1e5] * 3] * n, [[1, 0, 0, 0]] * n, ops, cols,
                [[1.0]] * n, [[i % 3] for i in range(n)], 3, cam)
    return sc, ops, cols


def _over(ops, cols, nblend):
    """Textbook over compositing of the first nblend flat layers."""
    T, c, s = 1.0, np.zeros(3), 0.0
    for o, col in zip(ops[:nblend], cols[:nblend]):
        c += np.asarray(col, np.float64) * o * T
        s += o * T
        T *= 1 - o
    return c, s, T


def test_transmittance_stop_flip_blends_the_crossing_layer():
    """T (1 - alpha_4) = t_min (1 - 5e-5): the fourth layer stops the walk by
    default (n = 3); the other outcome blends it (n = 4) and the fifth layer
    then stops the walk (T (1 - 0.5) < t_min)."""
    sc, ops, cols = _stop_scene(-5e-5)
    b = _branches(sc, [(3, 4)], nbits=1)
    assert b["nflag"][0, 0] == 1
    for j, nbl in ((0, 3), (1, 4)):
        c, s, T = _over(ops, cols, nbl)
        assert b["n_contrib"][0, j] == nbl
        assert np.allclose(b["rgb"][0, j], c, rtol=1e-9, atol=1e-12)
        assert math.isclose(b["sil"][0, j], s, rel_tol=1e-9)
        assert math.isclose(b["t_final"][0, j], T, rel_tol=1e-6)


def test_transmittance_stop_flip_stops_before_the_layer():
    """T (1 - alpha_4) = t_min (1 + 5e-5): blended by default (n = 4, the
    fifth layer stops it); the other outcome stops at the fourth (n = 3)."""
    sc, ops, cols = _stop_scene(5e-5)
    b = _branches(sc, [(0, 0)], nbits=1)
    assert b["n_contrib"][0, 0] == 4 and b["n_contrib"][0, 1] == 3
    c, s, T = _over(ops, cols, 3)
    assert np.allclose(b["rgb"][0, 1], c, rtol=1e-9, atol=1e-12)
    assert math.isclose(b["t_final"][0, 1], T, rel_tol=1e-6)


# ---------------------------------------------------------------- a flip is the moved threshold

def _grad_maps(rng, H, W, C):
    return {"rgb": rng.standard_normal((H, W, 3)), "depth": rng.standard_normal((H, W)),
            "sil": rng.standard_normal((H, W)), "sem": rng.standard_normal((H, W, C))}


def _flip_equals_moved_threshold(sc, branch, cfg_moved):
    cam = sc.cameras[0]
    cfg = O.config_array()
    arr = _arrays(sc)
    pr, mp = O.forward(arr, cam, cfg, sc.num_classes, branch=branch)
    pr2, mp2 = O.forward(arr, cam, cfg_moved, sc.num_classes)
    for key in ("rgb", "depth", "sil", "sem", "t_final", "n_contrib"):
        assert np.allclose(mp[key], mp2[key], rtol=1e-13, atol=1e-15), key
    dl = _grad_maps(np.random.default_rng(0), cam.height, cam.width, sc.num_classes)
    g1, _ = O.backward(arr, cam, cfg, sc.num_classes, dl, proj=pr, branch=branch)
    g2, _ = O.backward(arr, cam, cfg_moved, sc.num_classes, dl, proj=pr2)
    for key in g1:
        assert np.allclose(g1[key], g2[key], rtol=1e-12, atol=1e-15), key
    return mp


def test_alpha_flip_equals_cutoff_moved_below_alpha():
    """Taking the other outcome at every pixel where alpha sits just below
    alpha_min gives the maps and gradients of the plain definition with
    alpha_min moved just below that alpha (and no flagging)."""
    sc, alpha = _cutoff_scene(-3e-6)
    cam = sc.cameras[0]
    _, base = O.forward(_arrays(sc), cam, O.config_array(), sc.num_classes)
    branch = np.where(base["flags"] & 1, 1, 0).astype(np.uint32)
    assert int(branch.sum()) == 8  # the eight pixel centres at offsets (+-2.5, +-0.5), (+-0.5, +-2.5)
    moved = O.config_array(alpha_min=alpha * (1 - 1e-9), margin_alpha=0.0, margin_t=0.0)
    mp = _flip_equals_moved_threshold(sc, branch, moved)
    assert int(mp["n_contrib"].sum()) == int(base["n_contrib"].sum()) + 8


def test_stop_flip_equals_stop_moved_below_transmittance():
    """Blending the crossing layer everywhere equals the plain definition
    with t_min moved just below that layer's T (1 - alpha)."""
    sc, ops, _ = _stop_scene(-5e-5)
    cam = sc.cameras[0]
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, O.config_array())
    b = O.render_branches(pr, sc.opacity, sc.rgb, sc.sem_val, sc.sem_idx, sc.num_classes, cam, O.config_array(),
                          [(0, 0)], nbits=1)
    Tn = b["t_final"][0, 1]  # T after the crossing layer is blended
    branch = np.ones((cam.height, cam.width), np.uint32)
    moved = O.config_array(t_min=Tn * (1 - 1e-9), margin_alpha=0.0, margin_t=0.0)
    mp = _flip_equals_moved_threshold(sc, branch, moved)
    assert np.all(mp["n_contrib"] == 4)


# ---------------------------------------------------------------- invariants of every outcome

def test_every_outcome_keeps_the_compositing_invariants():
    """With wide margins many decisions are flagged; every enumerated outcome
    still satisfies S + T_final = 1 and sum_m P_m = S, branch 0 is the plain
    render, and outcomes differ only where a decision was flagged."""
    sc = scenes.tiny_scene(seed=3, n=600, width=24, height=20, f=20.0)
    cam = sc.cameras[0]
    cfg = O.config_array(margin_alpha=0.2, margin_t=0.5)
    pr, mp = O.forward(_arrays(sc), cam, cfg, sc.num_classes)
    ys, xs = np.nonzero(mp["flags"])
    assert len(ys) > 50
    pix = np.stack([xs, ys], 1)
    b = O.render_branches(pr, sc.opacity, sc.rgb, sc.sem_val, sc.sem_idx, sc.num_classes, cam, cfg, pix, nbits=3)
    assert np.abs(b["sil"] + b["t_final"] - 1).max() < 1e-12
    assert np.abs(b["sem"].sum(-1) - b["sil"]).max() < 1e-6
    for key in ("rgb", "sil", "sem", "t_final", "n_contrib"):
        assert np.array_equal(b[key][:, 0], mp[key][ys, xs]), key
    differs = np.any(b["n_contrib"] != b["n_contrib"][:, :1], axis=1)
    assert differs.mean() > 0.5
    assert np.all(b["nflag"][:, 0] >= 1)


# ---------------------------------------------------------------- the pixel rectangle

def _max_alpha_on_line(o, conic, mu, u, axis):
    """max over the other coordinate of o exp(-Q/2) on the line through
    pixel-centre coordinate u of `axis` (0: the column x = u, 1: the row
    y = u), by golden-section search of the convex quadratic Q (vectorised)."""
    a, b, c = conic[:, 0], conic[:, 1], conic[:, 2]
    d0 = u - mu[:, axis]
    lo = np.full_like(d0, -1e5)
    hi = np.full_like(d0, 1e5)

    def Q(t):
        dx, dy = (d0, t) if axis == 0 else (t, d0)
        return a * dx * dx + 2 * b * dx * dy + c * dy * dy

    r = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        x1, x2 = hi - r * (hi - lo), lo + r * (hi - lo)
        left = Q(x1) < Q(x2)  # the minimum lies in [lo, x2]
        hi = np.where(left, x2, hi)
        lo = np.where(left, lo, x1)
    qmin = Q(0.5 * (lo + hi))
    return o * np.exp(-0.5 * qmin)


def _check_tight(sc, cam, cfg):
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, cfg)
    vis = pr["visible"] == 1
    o = sc.opacity.astype(np.float64)[vis]
    conic, mu, rect = pr["conic"][vis], pr["mean2d"][vis], pr["rect"][vis]
    amin = O.ALPHA_MIN
    tol = 1e-9
    checked = 0
    for axis, (lo_i, hi_i, size) in enumerate(((0, 1, cam.width), (2, 3, cam.height))):
        lo, hi = rect[:, lo_i].astype(np.float64), rect[:, hi_i].astype(np.float64)
        inner_hi = _max_alpha_on_line(o, conic, mu, hi + 0.5, axis)
        outer_hi = _max_alpha_on_line(o, conic, mu, hi + 1.5, axis)
        inner_lo = _max_alpha_on_line(o, conic, mu, lo + 0.5, axis)
        outer_lo = _max_alpha_on_line(o, conic, mu, lo - 0.5, axis)
        # an edge not clamped to the image: its pixel-centre line reaches
        # alpha_min, the next line outward does not
        free_hi, free_lo = hi < size - 1, lo > 0
        assert np.all(inner_hi[free_hi] >= amin * (1 - tol)), axis
        assert np.all(outer_hi[free_hi] < amin * (1 + tol)), axis
        assert np.all(inner_lo[free_lo] >= amin * (1 - tol)), axis
        assert np.all(outer_lo[free_lo] < amin * (1 + tol)), axis
        # a clamped edge: the set reaches the image border line
        assert np.all(inner_hi[~free_hi] >= amin * (1 - tol)), axis
        assert np.all(inner_lo[~free_lo] >= amin * (1 - tol)), axis
        checked += int(free_hi.sum() + free_lo.sum())
    return checked


def test_rect_is_the_tight_box_of_the_cutoff_set():
    """Each rectangle edge is the outermost pixel-centre line that meets
    {o exp(-Q/2) >= alpha_min}: that line reaches alpha_min and the next one
    outward does not (maximum along the line found by golden-section search,
    not by the closed-form extent).  A looser box (e.g. 3 sigma) fails."""
    sc = scenes.tiny_scene(seed=1, n=600)
    rng = np.random.default_rng(5)
    sc.scales = (sc.scales * np.exp(rng.normal(0, 0.6, sc.scales.shape))).astype(np.float32)
    q = rng.standard_normal((sc.n, 4))
    sc.quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    n1 = _check_tight(sc, sc.cameras[0], O.config_array())
    n2 = _check_tight(sc, sc.cameras[0], O.config_array(lowpass=0.0))
    room = scenes.room_scene(n=20_000, targets=False)
    n3 = _check_tight(room, room.cameras[0], O.config_array())
    assert n1 > 500 and n2 > 500 and n3 > 5000


def test_far_mean_is_culled():
    """Reading: a projected mean 2^30 px or more from the image origin is
    culled even when its footprint would cover the image; just inside that
    range the same Gaussian covers the whole image."""
    cam = _cam(32, 32, 30.0)
    for x, visible in ((3.0e7, 1), (3.6e7, 0)):  # mean2d x = 30 x + 16: 9.0e8 and 1.08e9 (2^30 = 1.074e9)
        sc = _scene([[x, 0, 1.0]], [[6e7] * 3], [[1, 0, 0, 0]], [0.9], [[1, 1, 1]], [[1.0]], [[0]], 2, cam)
        pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, O.config_array())
        assert pr["visible"][0] == visible, x
        if visible:
            assert list(pr["rect"][0]) == [0, 31, 0, 31]
