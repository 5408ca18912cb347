"""The mapping loss fused into the forward launch (sgr_render_forward_loss),
against the FP64 loss oracle evaluated on the same rendered maps, and
against the unfused path (forward, loss-gradient kernel, backward)."""
import numpy as np
import pytest
import torch

from oracle import loss as OL
from paper_2506_00225_amd import Gaussians, loss_config, mapping_loss_grad, scenes

import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print("[case]", *a, flush=True)


def _scene(n=60_000, w=400, h=300, num_classes=102):
    sc = scenes.room_scene(seed=4, n=n, num_classes=num_classes, targets=False)
    cam = sc.cameras[0]
    sc.cameras = [scenes.Camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx - (cam.width - w) / 2,
                                cam.cy - (cam.height - h) / 2, w, h)]
    return sc


def _targets(rng, P, C, kind, k):
    t = {"rgb": rng.random((P, 3)).astype(np.float32), "depth": (rng.random(P) * 4.5 + 0.5).astype(np.float32)}
    if kind == "label":
        t["label"] = rng.integers(0, C, size=P).astype(np.int32)
    elif kind == "sem":
        # pseudo-ground truth: sharp for most pixels (entropy below ln k), flat for the rest
        conc = np.where(rng.random(P) < 0.8, 0.05, 5.0)[:, None]
        t["sem"] = np.stack([rng.dirichlet(np.ones(C) * c) for c in conc[:, 0]]).astype(np.float32)
    return t


@pytest.mark.parametrize("kind", ["label", "sem", "none"])
def test_fused_loss_matches_oracle_on_rendered_maps(kind):
    _say("fused loss vs oracle", kind)
    sc = _scene()
    cam = sc.cameras[0]
    P, C, k = cam.width * cam.height, sc.num_classes, sc.k
    rng = np.random.default_rng(7)
    tg = _targets(rng, P, C, kind, k)
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    fr.prepare(g)
    maps = fr.alloc_maps()
    grads, loss = fr.forward_loss(g, {kk: torch.from_numpy(v) for kk, v in tg.items()}, maps=maps)
    torch.cuda.synchronize()
    hw = (cam.height, cam.width)
    m = {"rgb": U.to_np(maps["rgb"]).reshape(*hw, 3), "depth": U.to_np(maps["depth"]).reshape(hw),
         "sil": U.to_np(maps["sil"]).reshape(hw), "sem": U.to_np(maps["sem"]).reshape(*hw, C)}
    t = {"rgb": tg["rgb"].reshape(*hw, 3), "depth": tg["depth"].reshape(hw)}
    if kind == "label":
        t["label"] = tg["label"].reshape(hw)
    if kind == "sem":
        t["sem"] = tg["sem"].reshape(*hw, C)
    want_loss, want, flags = OL.mapping_loss(m, t, C, k)
    assert float(loss[0]) == pytest.approx(want_loss, rel=1e-5)
    ok = ~flags
    for key, ch in (("rgb", 3), ("depth", 1), ("sil", 1), ("sem", C)):
        got = U.to_np(grads[key]).reshape(*hw, ch) if ch > 1 else U.to_np(grads[key]).reshape(hw)
        w = want[key]
        if ch > 1:
            got, w = got[ok], w[ok]
        else:
            got, w = got[ok], w[ok]
        scale = np.abs(w).max() + 1e-30
        assert np.allclose(got, w, rtol=1e-3, atol=1e-5 * scale), key
    print("flagged", int(flags.sum()), "of", P, flush=True)


def test_fused_loss_equals_unfused_cross_entropy_path():
    """Fused forward+loss then backward gives the gradients of forward,
    the separate loss-gradient kernel, and backward."""
    _say("fused vs unfused")
    sc = _scene(n=40_000, w=320, h=240)
    cam = sc.cameras[0]
    P, C = cam.width * cam.height, sc.num_classes
    rng = np.random.default_rng(8)
    tg = _targets(rng, P, C, "label", sc.k)
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    fr.prepare(g)
    maps = fr.forward(g)
    dl = mapping_loss_grad(maps, torch.from_numpy(tg["rgb"]).cuda(), torch.from_numpy(tg["depth"]).cuda(),
                           torch.from_numpy(tg["label"]).cuda(), C)
    ref = {kk: v.clone() for kk, v in fr.backward(g, dict(dl)).items()}
    fgr, loss = fr.forward_loss(g, {kk: torch.from_numpy(v) for kk, v in tg.items()})
    for key in ("rgb", "depth", "sil", "sem"):
        assert torch.allclose(fgr[key], dl[key], rtol=1e-6, atol=0), key
    got = fr.backward(g, dict(fgr))
    torch.cuda.synchronize()
    for key in ref:
        assert torch.allclose(got[key], ref[key], rtol=1e-5, atol=1e-12), key


def test_fused_loss_per_view_values_multiview():
    """Two views of different sizes in one launch: each view's loss and
    gradients equal those of the view rendered alone."""
    _say("fused multiview")
    sc = _scene(n=30_000, w=256, h=192)
    cam = sc.cameras[0]
    cam2 = scenes.Camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx + 30, cam.cy - 10, 200, 150)
    cams = [cam, cam2]
    rng = np.random.default_rng(9)
    tgs = [_targets(rng, c.width * c.height, sc.num_classes, "sem", sc.k) for c in cams]
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc, cams=cams)
    fr.prepare(g)
    grads, loss = fr.forward_loss(g, [{kk: torch.from_numpy(v) for kk, v in t.items()} for t in tgs])
    torch.cuda.synchronize()
    for v, c in enumerate(cams):
        f1 = U.frame_for(sc, cams=[c])
        f1.prepare(g)
        g1, l1 = f1.forward_loss(g, {kk: torch.from_numpy(x) for kk, x in tgs[v].items()})
        torch.cuda.synchronize()
        assert float(l1[0]) == float(loss[v])
        for key in g1:
            assert torch.equal(fr.split(grads[key])[v].reshape(-1), g1[key].reshape(-1)), (v, key)


def _same_sem_grad(dense_g, sparse_g, mag):
    """Top-k value gradients of the one-class kernel against the dense one.
    With the semantic loss kept off geometry (k = 16, C <= 128) the one-class
    kernel sums each key's semantic values in per-wave LDS bins, lane by
    lane, where the dense kernel sums them in a tree over the wave: the same
    terms in another order, so equal to float32 summation error, at most 64
    unit roundoffs of the sum of the terms' magnitudes (`mag`, the same
    gradient for |dL/dsem|)."""
    d = (dense_g.double() - sparse_g.double()).abs()
    bound = 64 * 2.0 ** -24 * mag.double().abs() + 1e-30
    assert bool((d <= bound).all()), (float((d - bound).max()), int((d > bound).sum()))


def test_sparse_semantic_gradient_equals_dense():
    """One (class, value) per pixel in registers gives the bits of the same
    gradient written out densely and staged in LDS (the top-k value
    gradients of the ranked one-class kernel to float32 summation order, see
    _same_sem_grad); the fused loss's sparse output gives the bits of its
    dense output."""
    _say("sparse semantic gradient")
    sc = _scene(n=50_000, w=320, h=240)
    cam = sc.cameras[0]
    P, C = cam.width * cam.height, sc.num_classes
    rng = np.random.default_rng(10)
    g = Gaussians.from_scene(sc)
    for semgeo in (0, 1):
        fr = U.frame_for(sc, semgeo=semgeo)
        fr.prepare(g)
        fr.forward(g)
        lab = rng.integers(-1, C, size=P).astype(np.int32)  # -1: no semantic gradient at that pixel
        val = rng.standard_normal(P).astype(np.float32)
        dense = np.zeros((P, C), np.float32)
        ok = lab >= 0
        dense[np.nonzero(ok)[0], lab[ok]] = val[ok]
        base = {"rgb": torch.randn(P, 3, device="cuda"), "depth": torch.randn(P, device="cuda"),
                "sil": torch.randn(P, device="cuda")}
        gd = {k: v.clone() for k, v in fr.backward(g, dict(base, sem=torch.from_numpy(dense).cuda())).items()}
        mag = fr.backward(g, dict(base, sem=torch.from_numpy(np.abs(dense)).cuda()))["sem_val"].clone()
        gs = fr.backward(g, dict(base, sem_label=torch.from_numpy(lab).cuda(), sem_at_label=torch.from_numpy(val).cuda()))
        torch.cuda.synchronize()
        for k in gd:
            if k == "sem_val" and semgeo == 0:
                _same_sem_grad(gd[k], gs[k], mag)
            else:
                assert torch.equal(gd[k], gs[k]), (semgeo, k)
    # fused loss: sparse output == dense output, and the backward agrees bitwise
    tg = _targets(rng, P, C, "label", sc.k)
    fr = U.frame_for(sc)
    fr.prepare(g)
    tt = {kk: torch.from_numpy(v) for kk, v in tg.items()}
    gdn, l1 = fr.forward_loss(g, tt)
    ref = {k: v.clone() for k, v in fr.backward(g, dict(gdn)).items()}
    mag = fr.backward(g, dict(gdn, sem=gdn["sem"].abs()))["sem_val"].clone()
    gsp, l2 = fr.forward_loss(g, tt, sparse_sem=True)
    got = fr.backward(g, dict(gsp))
    torch.cuda.synchronize()
    assert float(l1[0]) == float(l2[0])
    lab = torch.from_numpy(tg["label"]).cuda().long()
    assert torch.equal(gdn["sem"].gather(1, lab[:, None])[:, 0], gsp["sem_at_label"])
    for k in ref:
        if k == "sem_val":
            _same_sem_grad(ref[k], got[k], mag)
        else:
            assert torch.equal(ref[k], got[k]), k


def test_label_only_lookup_with_repeated_classes():
    """The label-only forward finds the label's value through a class mask
    when an entry's classes are distinct and walks the list otherwise:
    with 30 % of the top-k lists carrying a repeated class, loss, maps and
    gradients still equal, bit for bit, those of the launch with all C class
    sums."""
    _say("label-only lookup, repeated classes")
    sc = _scene(n=40_000, w=256, h=192, num_classes=102)
    rng = np.random.default_rng(12)
    dup = rng.random(sc.n) < 0.3
    sc.sem_idx[dup, 3] = sc.sem_idx[dup, 0]
    cam = sc.cameras[0]
    tgs = [{kk: torch.from_numpy(v) for kk, v in _targets(rng, cam.width * cam.height, 102, "label", sc.k).items()}]
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    fr.prepare(g)
    keys = ("rgb", "depth", "sil", "t_final", "n_contrib")
    m1 = {kk: v for kk, v in fr.alloc_maps().items() if kk in keys}
    g1, l1 = fr.forward_loss(g, tgs, maps=m1, sparse_sem=True)
    g1 = {kk: v.clone() for kk, v in g1.items()}
    l1 = l1.clone()
    m2 = fr.alloc_maps()
    g2, l2 = fr.forward_loss(g, tgs, maps=m2, sparse_sem=True)
    torch.cuda.synchronize()
    assert torch.equal(l1, l2)
    for kk in g1:
        assert torch.equal(g1[kk], g2[kk]), kk
    for kk in m1:
        assert torch.equal(m1[kk], m2[kk]), kk
    assert fr.status()[0] == 0


@pytest.mark.parametrize("C", [102, 256])
def test_label_only_class_sums_equal_full_path(C):
    """With cross-entropy targets and no semantic map asked for, the fused
    forward keeps only each pixel's class sum at its label.  Loss, maps and
    gradients equal, bit for bit, those of the launch that accumulates all C
    class sums (asked for the semantic map as well); two views of different
    sizes, one with a label outside [0, C) reported as an input error; the
    loss also matches the oracle on the rendered maps."""
    _say("label-only class sums", C)
    sc = _scene(n=40_000, w=256, h=192, num_classes=C)
    cam = sc.cameras[0]
    cams = [cam, scenes.Camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx + 20, cam.cy - 10, 200, 150)]
    rng = np.random.default_rng(11)
    tgs = [{kk: torch.from_numpy(v) for kk, v in _targets(rng, c.width * c.height, C, "label", sc.k).items()}
           for c in cams]
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc, cams=cams)
    fr.prepare(g)
    keys = ("rgb", "depth", "sil", "t_final", "n_contrib")
    m1 = {kk: v for kk, v in fr.alloc_maps().items() if kk in keys}
    g1, l1 = fr.forward_loss(g, tgs, maps=m1, sparse_sem=True)         # label-only sums
    g1 = {kk: v.clone() for kk, v in g1.items()}
    l1 = l1.clone()
    m2 = fr.alloc_maps()
    g2, l2 = fr.forward_loss(g, tgs, maps=m2, sparse_sem=True)         # all C sums (sem map asked for)
    torch.cuda.synchronize()
    assert torch.equal(l1, l2)
    for kk in g1:
        assert torch.equal(g1[kk], g2[kk]), kk
    for kk in m1:
        assert torch.equal(m1[kk], m2[kk]), kk
    st, _, _ = fr.status()
    assert st == 0
    # the oracle's loss on the maps of view 0
    hw = (cam.height, cam.width)
    P0 = cam.width * cam.height
    m = {"rgb": U.to_np(m2["rgb"][:P0]).reshape(*hw, 3), "depth": U.to_np(m2["depth"][:P0]).reshape(hw),
         "sil": U.to_np(m2["sil"][:P0]).reshape(hw), "sem": U.to_np(m2["sem"][:P0]).reshape(*hw, C)}
    t = {"rgb": U.to_np(tgs[0]["rgb"]).reshape(*hw, 3), "depth": U.to_np(tgs[0]["depth"]).reshape(hw),
         "label": U.to_np(tgs[0]["label"]).reshape(hw)}
    want_loss, _, _ = OL.mapping_loss(m, t, C, sc.k)
    assert float(l1[0]) == pytest.approx(want_loss, rel=1e-5)
    # a label outside [0, C): status SGR_EINVAL, no loss term for that pixel
    bad = [dict(tg) for tg in tgs]
    bad[1]["label"] = bad[1]["label"].clone()
    bad[1]["label"][7] = C
    fr.forward_loss(g, bad, sparse_sem=True)
    torch.cuda.synchronize()
    st, _, _ = fr.status()
    assert st == 1
