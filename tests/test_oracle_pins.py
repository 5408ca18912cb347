"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms of a single Gaussian, textbook "over" compositing worked by hand,
invariants implied by Eq. 1 / Eq. 3, brute force, central finite
differences, and library entropy.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_00225_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scene(means, scales, quats, opacity, rgb, sem_val, sem_idx, C, cam):
    f = lambda a: np.asarray(a, dtype=np.float32)
    return scenes.Scene(f(means), f(scales), f(quats), f(opacity), f(rgb), f(sem_val),
                        np.asarray(sem_idx, dtype=np.uint8), C, [cam])


def _cam(w, h, f, R=None, t=None, cx=None, cy=None):
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    t = np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32)
    return scenes.Camera(R, t, f, f, w / 2 if cx is None else cx, h / 2 if cy is None else cy, w, h)


def _fwd(sc, cfg=None, brute=False):
    cfg = O.config_array() if cfg is None else cfg
    return O.forward(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes, brute=brute)


# ---------------------------------------------------------------- closed forms

def test_single_isotropic_on_axis_closed_form():
    """Eq. 1 with one Gaussian: C = c a, D = z a, S = a, P_m = v_m a,
    T = 1 - a, where a = min(0.99, o exp(-r^2 / (2 (f^2 s^2 / z^2 + l))))."""
    f, z, s, o, lp = 30.0, 2.0, 0.05, 0.8, O.LOWPASS
    cam = _cam(32, 32, f)
    sc = _scene([[0, 0, z]], [[s, s, s]], [[1, 0, 0, 0]], [o], [[0.2, 0.5, 0.9]], [[0.7, 0.3]], [[1, 3]], 4, cam)
    pr, mp = _fwd(sc)
    s32, o32, z32 = float(np.float32(s)), float(np.float32(o)), float(np.float32(z))
    var = (f * s32 / z32) ** 2 + lp
    assert np.allclose(pr["cov2d"][0], [var, 0.0, var], rtol=1e-13, atol=1e-15)
    assert np.allclose(pr["conic"][0], [1 / var, 0.0, 1 / var], rtol=1e-13, atol=1e-15)
    assert np.allclose(pr["mean2d"][0], [16.0, 16.0], rtol=0, atol=1e-12)
    ys, xs = np.mgrid[0:32, 0:32]
    r2 = (xs + 0.5 - 16.0) ** 2 + (ys + 0.5 - 16.0) ** 2
    a = np.minimum(O.ALPHA_MAX, o32 * np.exp(-r2 / (2 * var)))
    a = np.where(a >= O.ALPHA_MIN, a, 0.0)
    c = np.float32([0.2, 0.5, 0.9]).astype(np.float64)
    v = np.float32([0.7, 0.3]).astype(np.float64)
    assert np.allclose(mp["rgb"], a[..., None] * c, atol=1e-14)
    assert np.allclose(mp["depth"], a * z32, atol=1e-14)
    assert np.allclose(mp["sil"], a, atol=1e-14)
    assert np.allclose(mp["t_final"], 1 - a, atol=1e-14)
    assert np.allclose(mp["sem"][..., 1], a * v[0], atol=1e-14)
    assert np.allclose(mp["sem"][..., 3], a * v[1], atol=1e-14)
    assert np.all(mp["sem"][..., [0, 2]] == 0)
    assert np.array_equal(mp["n_contrib"], (a > 0).astype(np.int32))


def test_single_isotropic_off_axis_closed_form():
    """Off axis, Sigma2 = s^2 J J^T + l I with J the perspective Jacobian
    [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]] written out by hand."""
    f, s = 50.0, 0.04
    x, y, z = 0.3, -0.2, 2.5
    cam = _cam(64, 48, f)
    sc = _scene([[x, y, z]], [[s] * 3], [[1, 0, 0, 0]], [0.6], [[1, 1, 1]], [[1.0]], [[0]], 2, cam)
    pr, _ = _fwd(sc)
    x, y, z, s = (float(np.float32(v)) for v in (x, y, z, s))
    jj_xx = f * f / z ** 2 + f * f * x * x / z ** 4
    jj_xy = f * f * x * y / z ** 4
    jj_yy = f * f / z ** 2 + f * f * y * y / z ** 4
    want = [s * s * jj_xx + O.LOWPASS, s * s * jj_xy, s * s * jj_yy + O.LOWPASS]
    assert np.allclose(pr["cov2d"][0], want, rtol=1e-12)
    assert np.allclose(pr["mean2d"][0], [f * x / z + 32, f * y / z + 24], rtol=1e-14)


def test_anisotropic_rotated_about_optical_axis():
    """Scales (s1, s2, s3) rotated by theta about the optical axis (quaternion
    (cos theta/2, 0, 0, sin theta/2)): on the axis Sigma2 = (f/z)^2 R(theta)
    diag(s1^2, s2^2) R(theta)^T + l I."""
    f, z, th = 40.0, 3.0, 0.7
    s1, s2, s3 = 0.05, 0.02, 0.3
    cam = _cam(64, 64, f)
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    sc = _scene([[0, 0, z]], [[s1, s2, s3]], [q], [0.9], [[1, 1, 1]], [[1.0]], [[0]], 2, cam)
    pr, _ = _fwd(sc)
    q32 = np.float32(q).astype(np.float64)
    th = 2 * math.atan2(q32[3], q32[0])
    s1, s2 = float(np.float32(s1)), float(np.float32(s2))
    c_, s_ = math.cos(th), math.sin(th)
    k2 = (f / z) ** 2
    want = [k2 * (c_ * c_ * s1 * s1 + s_ * s_ * s2 * s2) + O.LOWPASS,
            k2 * c_ * s_ * (s1 * s1 - s2 * s2),
            k2 * (s_ * s_ * s1 * s1 + c_ * c_ * s2 * s2) + O.LOWPASS]
    assert np.allclose(pr["cov2d"][0], want, rtol=1e-6)


def test_camera_pose_projection_by_hand():
    """Room keyframe at (5, 4, 1.5) looking along +x (camera x = -y_w,
    y = -z_w, z = +x_w): the world point (7, 3, 1) sits at camera (1, 0.5, 2),
    so it projects to (600*1/2 + 600, 600*0.5/2 + 340) = (900, 490)."""
    cam = scenes.room_view_camera()
    sc = _scene([[7, 3, 1]], [[0.02] * 3], [[1, 0, 0, 0]], [0.5], [[1, 1, 1]], [[1.0]], [[0]], 2, cam)
    pr, _ = _fwd(sc)
    assert np.allclose(pr["pcam"][0], [1.0, 0.5, 2.0], atol=1e-12)
    assert np.allclose(pr["mean2d"][0], [900.0, 490.0], atol=1e-9)
    assert pr["visible"][0] == 1


# ---------------------------------------------------------------- compositing by hand

def _flat(depths, opac, colours, C=3, w=8, h=8):
    """Huge flat Gaussians on the axis: alpha = o to within 1e-10 everywhere."""
    n = len(depths)
    cam = _cam(w, h, 8.0)
    sem_idx = [[i % C] for i in range(n)]
    return _scene([[0, 0, d] for d in depths], [[1e5] * 3] * n, [[1, 0, 0, 0]] * n, opac, colours,
                  [[1.0]] * n, sem_idx, C, cam)


def test_over_compositing_golden():
    """Worked textbook over-compositing (Eq. 1), values in tests/golden."""
    with open(os.path.join(GOLDEN, "over_compositing.json")) as fh:
        gold = json.load(fh)
    for case in gold["cases"]:
        sc = _flat(case["depths"], case["opacity"], case["rgb"])
        _, mp = _fwd(sc)
        for key in ("rgb", "depth", "sil", "t_final"):
            assert np.allclose(mp[key], np.broadcast_to(case["expect"][key], mp[key].shape), atol=1e-8), key
        assert np.all(mp["n_contrib"] == case["expect"]["n_contrib"])


def test_transmittance_stop_excludes_crossing_gaussian():
    """20 flat o=0.5 layers: T after n blends is 2^-n; 2^-14 < 1e-4 so the
    14th layer is not blended: n_contrib = 13, T = 2^-13."""
    n = 20
    sc = _flat([1.0 + 0.1 * i for i in range(n)], [0.5] * n, [[1, 1, 1]] * n)
    _, mp = _fwd(sc)
    assert np.all(mp["n_contrib"] == 13)
    assert np.allclose(mp["t_final"], 2.0 ** -13, rtol=1e-8)
    assert np.allclose(mp["sil"], 1 - 2.0 ** -13, rtol=1e-8)
    assert np.allclose(mp["rgb"], (1 - 2.0 ** -13), rtol=1e-8)


def test_alpha_clamp_and_cutoff():
    """o = 0.999 is clamped to alpha_max; a second such layer would take T
    to (1 - 0.99)^2 < 1e-4 and is not blended.  o below 1/255 is culled."""
    sc = _flat([1.0, 2.0], [0.999, 0.999], [[1, 0, 0], [0, 1, 0]])
    _, mp = _fwd(sc)
    amax = O.ALPHA_MAX
    assert np.all(mp["n_contrib"] == 1)
    assert np.allclose(mp["rgb"][..., 0], amax, atol=1e-9)
    assert np.allclose(mp["t_final"], 1 - amax, atol=1e-9)
    sc = _flat([1.0], [0.0039], [[1, 1, 1]])
    pr, mp = _fwd(sc)
    assert pr["visible"][0] == 0
    assert np.all(mp["n_contrib"] == 0) and np.all(mp["t_final"] == 1.0) and np.all(mp["sem"] == 0)


def test_depth_order_not_id_order_and_id_tiebreak():
    """Sorting is by camera-space depth; equal fp32 depths keep id order."""
    sc = _flat([3.0, 2.0, 1.0], [0.5] * 3, [[0, 0, 1], [0, 1, 0], [1, 0, 0]])
    _, mp = _fwd(sc)
    assert np.allclose(mp["rgb"][0, 0], [0.5, 0.25, 0.125], atol=1e-8)
    sc = _flat([2.0, 2.0], [0.5, 0.5], [[1, 0, 0], [0, 1, 0]])
    _, mp = _fwd(sc)
    assert np.allclose(mp["rgb"][0, 0], [0.5, 0.25, 0.0], atol=1e-8)


# ---------------------------------------------------------------- invariants and brute force

@pytest.mark.parametrize("lowpass", [0.0, O.LOWPASS])
def test_invariants_tiny_scene(lowpass):
    sc = scenes.tiny_scene()
    cfg = O.config_array(lowpass=lowpass)
    pr, mp = _fwd(sc, cfg)
    assert np.abs(mp["sil"] + mp["t_final"] - 1).max() < 1e-12
    # top-k values sum to 1 in float32: semantic mass equals silhouette up to k ulp
    assert np.abs(mp["sem"].sum(-1) - mp["sil"]).max() < 1e-6
    assert mp["t_final"].min() >= O.T_MIN
    assert mp["rgb"].min() >= 0 and mp["rgb"].max() <= 1
    zmax = pr["depth"][pr["visible"] == 1].max()
    assert np.all(mp["depth"] <= zmax * mp["sil"] + 1e-12)
    assert np.array_equal(mp["n_contrib"] == 0, mp["sil"] == 0)


def test_brute_force_equals_row_lists():
    """Candidate lists from pixel rectangles change nothing: brute force over
    every visible Gaussian gives bit-identical maps."""
    for seed in range(3):
        sc = scenes.tiny_scene(seed=seed, n=400, width=24, height=20, f=20.0)
        _, a = _fwd(sc)
        _, b = _fwd(sc, brute=True)
        for key in ("rgb", "depth", "sil", "sem", "t_final", "n_contrib"):
            assert np.array_equal(a[key], b[key]), key


def test_rect_contains_every_pixel_above_cutoff():
    """Every pixel where o exp(-Q/2) >= alpha_min lies inside the Gaussian's
    pixel rectangle (checked over the whole image for each Gaussian)."""
    sc = scenes.tiny_scene(seed=1, n=300)
    cam = sc.cameras[0]
    pr, _ = _fwd(sc)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    for i in range(sc.n):
        if not np.any(pr["conic"][i]):
            continue
        a, b, c = pr["conic"][i]
        dx = xs + 0.5 - pr["mean2d"][i, 0]
        dy = ys + 0.5 - pr["mean2d"][i, 1]
        al = float(sc.opacity[i]) * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        hit = al >= O.ALPHA_MIN
        if not hit.any():
            continue
        assert pr["visible"][i] == 1
        r = pr["rect"][i]
        assert xs[hit].min() >= r[0] and xs[hit].max() <= r[1]
        assert ys[hit].min() >= r[2] and ys[hit].max() <= r[3]


def test_reference_keys_brute_force():
    """The key list equals a plain loop over (Gaussian, tile) pairs."""
    sc = scenes.tiny_scene(seed=2, n=500)
    cam = sc.cameras[0]
    pr, _ = _fwd(sc)
    keys, ranges, off = O.reference_keys([pr], [cam], 16, 16)
    txn = (cam.width + 15) // 16
    want = []
    for i in range(sc.n):
        if not pr["visible"][i]:
            continue
        r = pr["rect"][i]
        for ty in range(r[2] // 16, r[3] // 16 + 1):
            for tx in range(r[0] // 16, r[1] // 16 + 1):
                want.append((0, ty * txn + tx, int(pr["zbits"][i]), i))
    want.sort()
    assert np.array_equal(keys, np.array(want, np.int64))
    for t in range(ranges.shape[0]):
        s, e = ranges[t]
        assert np.all(keys[s:e, 1] == t)
        assert (keys[:, 1] == t).sum() == e - s


# ---------------------------------------------------------------- gradients vs finite differences

def _grad_scene(seed, n=24, w=20, h=16, C=6, k=3):
    rng = np.random.default_rng(100 + seed)
    f = 18.0
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.5, 0.5, n), rng.uniform(1.0, 2.0, n)], 1)
    scales = np.exp(rng.normal(math.log(0.12), 0.4, (n, 3)))
    quats = rng.standard_normal((n, 4)) * np.array([1, 1, 1, 1])
    quats *= 1.3  # unnormalised on purpose: project normalises
    opacity = rng.uniform(0.2, 0.95, n)
    rgb = rng.random((n, 3))
    sem_idx = np.argsort(rng.random((n, C)), 1)[:, :k]
    sem_val = rng.dirichlet(np.ones(k), n)
    cam = _cam(w, h, f)
    sc = _scene(means, scales, quats, opacity, rgb, sem_val, sem_idx, C, cam)
    grads = {"rgb": rng.standard_normal((h, w, 3)), "depth": rng.standard_normal((h, w)),
             "sil": rng.standard_normal((h, w)), "sem": rng.standard_normal((h, w, C))}
    return sc, grads


def _compare(analytic, fd, name, rtol=1e-5):
    ok = ~np.isnan(fd)
    assert ok.mean() > 0.9, f"{name}: too many coordinates straddle a decision"
    a, b = analytic[ok], fd[ok]
    scale = np.sqrt(np.mean(b * b)) + 1e-30
    err = np.abs(a - b)
    assert np.all(err <= rtol * np.abs(b) + 1e-5 * scale), (name, float(err.max()), float(scale))


@pytest.mark.parametrize("seed", [0, 1])
def test_analytic_gradient_matches_finite_differences_semgeo(seed):
    """With sem_grad_to_geometry = 1 the analytic gradient is the exact
    gradient of the whole loss, so every parameter matches central FD."""
    sc, grads = _grad_scene(seed)
    cfg = O.config_array(sem_grad_to_geometry=1)
    g, _ = O.backward(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes, grads)
    fd = O.finite_difference(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes, grads)
    for name in fd:
        _compare(g[name], fd[name], name)


def test_semantic_gradient_isolated_from_geometry():
    """With sem_grad_to_geometry = 0 (Sec. 3.1: the semantic loss only
    updates semantic attributes) geometry gradients equal FD of the loss with
    the semantic term removed, while semantic values still see the full loss."""
    sc, grads = _grad_scene(3)
    cfg = O.config_array(sem_grad_to_geometry=0)
    g, _ = O.backward(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes, grads)
    nosem = dict(grads, sem=np.zeros_like(grads["sem"]))
    fd_geo = O.finite_difference(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes, nosem,
                                 params=("means", "scales", "quats", "opacity", "rgb"))
    for name in fd_geo:
        _compare(g[name], fd_geo[name], name)
    fd_sem = O.finite_difference(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes, grads,
                                 params=("sem_val",))
    _compare(g["sem_val"], fd_sem["sem_val"], "sem_val")


def test_single_gaussian_gradient_closed_forms():
    """One Gaussian: dC/dc = alpha, dS/do = G where unclamped, and a pixel
    where alpha is clamped passes no gradient to opacity."""
    f, z, s, o = 30.0, 2.0, 0.05, 0.8
    cam = _cam(32, 32, f)
    sc = _scene([[0, 0, z]], [[s] * 3], [[1, 0, 0, 0]], [o], [[0.2, 0.5, 0.9]], [[1.0]], [[0]], 2, cam)
    pr, mp = _fwd(sc)
    zero = {"rgb": np.zeros((32, 32, 3)), "depth": np.zeros((32, 32)), "sil": np.zeros((32, 32)),
            "sem": np.zeros((32, 32, 2))}
    g = dict(zero, rgb=np.ones((32, 32, 3)))
    _, g2 = O.backward(O.scene_arrays(sc), cam, O.config_array(), 2, g)
    alpha_sum = mp["sil"].sum()
    assert np.allclose(g2["rgb"][0], [alpha_sum] * 3, rtol=1e-12)
    g = dict(zero, sil=np.ones((32, 32)))
    _, g2 = O.backward(O.scene_arrays(sc), cam, O.config_array(), 2, g)
    o32 = float(np.float32(o))
    assert np.isclose(g2["opacity"][0], alpha_sum / o32, rtol=1e-12)


# ---------------------------------------------------------------- scoring

def test_score_empty_scene_and_uniform():
    """No Gaussian: every pixel empty and H = ln C (clip makes it uniform)."""
    C = 7
    maps = {"sem": np.zeros((5, 6, C)), "n_contrib": np.zeros((5, 6), np.int32)}
    r = O.score(maps, C)
    assert r["n_empty"] == 30
    assert math.isclose(r["entropy_sum"], 30 * math.log(C), rel_tol=1e-13)


def test_score_one_hot_closed_form():
    """P = e_0: q = (1, 0.001, ...) / Z with Z = 1 + 0.001 (C - 1)."""
    C = 102
    sem = np.zeros((1, 1, C))
    sem[..., 0] = 1.0
    r = O.score({"sem": sem, "n_contrib": np.ones((1, 1), np.int32)}, C)
    Z = 1 + 0.001 * (C - 1)
    want = -(1 / Z) * math.log(1 / Z) - (C - 1) * (0.001 / Z) * math.log(0.001 / Z)
    assert math.isclose(r["entropy_sum"], want, rel_tol=1e-13)
    assert r["n_empty"] == 0


def test_score_matches_scipy_entropy():
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(5)
    C = 40
    sem = rng.random((6, 9, C)) * (rng.random((6, 9, C)) < 0.3) * 0.2
    nc = rng.integers(0, 3, (6, 9)).astype(np.int32)
    r = O.score({"sem": sem, "n_contrib": nc}, C)
    q = np.clip(sem, 0.001, 1.0)
    want = scipy_stats.entropy(q.reshape(-1, C), axis=1).sum()
    assert math.isclose(r["entropy_sum"], want, rel_tol=1e-12)
    assert r["n_empty"] == int((nc == 0).sum())
