"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: tile keys, sort order and ranges bit-exact; maps within 1e-4 absolute
and n_contrib exact on pixels where no decision sits within the oracle's
margin of a threshold; gradients within 1e-3 relative.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_00225_amd import Frame, Gaussians, SgrError, autotune, make_config, render, scenes, score_maps

import gpu_util as U

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00225_amd import _lib
    _lib.lib()


def _room_crop(n=200_000, w=1200, h=680, seed=0):
    sc = scenes.room_scene(seed=seed, n=n, targets=False)
    cam = sc.cameras[0]
    if (w, h) != (cam.width, cam.height):
        cam = scenes.Camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx - (cam.width - w) / 2, cam.cy - (cam.height - h) / 2,
                            w, h)
        sc.cameras = [cam]
    return sc


# ---------------------------------------------------------------- projection and binning

@pytest.mark.parametrize("case", ["tiny", "room_crop", "tiny_lowpass0"])
def test_project_and_keys_bit_exact(case):
    _say("project/keys", case)
    lowpass = 0.0 if case == "tiny_lowpass0" else None
    sc = scenes.tiny_scene() if case.startswith("tiny") else _room_crop(n=50_000, w=400, h=300)
    fr = U.frame_for(sc, lowpass=lowpass)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    torch.cuda.synchronize()
    cfg = U.oracle_cfg(lowpass=lowpass)
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, sc.cameras[0], cfg)
    gp = U.gpu_proj(fr)
    vis = pr["visible"] == 1
    assert np.array_equal(gp["visible"], vis)
    assert np.array_equal(gp["zbits"], pr["zbits"])
    assert np.array_equal(gp["rect"][vis], pr["rect"][vis])
    assert np.array_equal(gp["count"][vis], U.tiles_touched(pr["rect"][vis]))
    assert np.allclose(gp["mean2d"][vis], pr["mean2d"][vis], rtol=0, atol=2e-6)
    assert np.allclose(gp["conic"][vis], pr["conic"][vis], rtol=2e-6, atol=1e-12)
    keys, rng = U.gpu_keys(fr)
    want, wrng, _ = O.reference_keys([pr], sc.cameras)
    assert keys.shape == want.shape
    assert np.array_equal(keys, want)
    assert np.array_equal(rng, wrng)


def test_multiview_keys_bit_exact():
    _say("multiview keys")
    sc = scenes.candidate_scene(n=20_000, nviews=5)
    fr = U.frame_for(sc)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    torch.cuda.synchronize()
    cfg = U.oracle_cfg()
    prs = [O.project(sc.means, sc.scales, sc.quats, sc.opacity, c, cfg) for c in sc.cameras]
    keys, rng = U.gpu_keys(fr)
    want, wrng, _ = O.reference_keys(prs, sc.cameras)
    assert np.array_equal(keys, want)
    assert np.array_equal(rng, wrng)


def test_keys_bit_exact_past_the_small_sort_limits():
    """Eight views of 150k Gaussians (1.2M pairs): past 512 compaction
    workgroups (the per-block visible counts are scanned rather than summed
    by each workgroup) and past the small-sort form of the depth sort (its
    counts scanned, blocks of 2048); keys, order and ranges still equal the
    oracle's bit for bit."""
    _say("keys past the small sort limits")
    sc = scenes.candidate_scene(n=150_000, nviews=8)
    assert sc.n * len(sc.cameras) > 512 * 2048
    fr = U.frame_for(sc)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    torch.cuda.synchronize()
    st, nvis, _ = fr.status()
    assert st == 0
    cfg = U.oracle_cfg()
    prs = [O.project(sc.means, sc.scales, sc.quats, sc.opacity, c, cfg) for c in sc.cameras]
    assert nvis == sum(int(p["visible"].sum()) for p in prs)
    keys, rng = U.gpu_keys(fr)
    want, wrng, _ = O.reference_keys(prs, sc.cameras)
    assert np.array_equal(keys, want)
    assert np.array_equal(rng, wrng)


# ---------------------------------------------------------------- forward

def _forward_case(sc, lowpass=None):
    fr = U.frame_for(sc, lowpass=lowpass)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    maps = fr.forward(g)
    torch.cuda.synchronize()
    got = {k: fr.split(v)[0].cpu().numpy() for k, v in maps.items()}
    view = U.OracleView.of_scene(sc, cfg=U.oracle_cfg(lowpass=lowpass))
    return fr, got, view.pr, view


@pytest.mark.parametrize("seed", [0, 1])
def test_forward_tiny_scene(seed):
    _say("forward tiny", seed)
    sc = scenes.tiny_scene(seed=seed)
    _, got, _, view = _forward_case(sc)
    rep = U.compare_maps(got, view)
    assert rep["flagged"] <= 10 and rep["unresolved"] == 0, rep


def test_forward_ragged_view_and_brute_force():
    """A 70x45 view (ragged tiles on both axes) against the brute-force
    oracle (no rectangles, no binning)."""
    _say("forward ragged brute")
    sc = scenes.tiny_scene(seed=3, n=1500, width=70, height=45, f=50.0)
    fr, got, pr, view = _forward_case(sc)
    _, brute = O.forward(O.scene_arrays(sc), sc.cameras[0], U.oracle_cfg(), sc.num_classes, brute=True)
    for key in ("rgb", "depth", "sil", "sem", "t_final", "n_contrib", "flags"):
        assert np.array_equal(brute[key], view.mp[key]), key
    rep = U.compare_maps(got, view)
    assert rep["unresolved"] == 0, rep


def test_forward_thin_rotated_gaussians():
    """Needle-like Gaussians (one long axis, random rotations) whose pixel
    rectangles mostly miss the ellipse: the per-block ellipse cull must
    never drop a blend.  Maps and n_contrib against the oracle, and the
    backward against the oracle's gradient."""
    _say("forward thin rotated")
    sc = scenes.tiny_scene(seed=21, n=1500, width=96, height=80, f=70.0)
    rng = np.random.default_rng(22)
    long_axis = rng.integers(0, 3, sc.n)
    sc.scales[:] = np.float32(0.004)
    sc.scales[np.arange(sc.n), long_axis] = rng.uniform(0.05, 0.4, sc.n).astype(np.float32)
    q = rng.standard_normal((sc.n, 4))
    sc.quats[:] = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    sc.opacity[:] = rng.uniform(0.3, 0.99, sc.n).astype(np.float32)
    fr, got, pr, view = _forward_case(sc)
    rep = U.compare_maps(got, view)
    assert rep["flagged"] <= 20 and rep["unresolved"] == 0, rep
    assert int(view.mp["n_contrib"].sum()) > 20 * sc.cameras[0].width  # the needles do overlap pixels
    _backward_case(sc, 0)


def test_forward_room_full_frame():
    """200k Gaussians in the room at 1200x680 (the forward+backward workload)."""
    _say("forward room 200k 1200x680")
    sc = _room_crop()
    fr, got, pr, view = _forward_case(sc)
    rep = U.compare_maps(got, view)
    assert rep["flagged"] <= 0.002 * view.flags.size and rep["unresolved"] == 0, rep
    print("forward room report", rep, flush=True)
    s = got["sil"].astype(np.float64) + got["t_final"]
    assert np.abs(s - 1).max() < 2e-5
    assert (got["sem"].sum(-1) - got["sil"]).__abs__().max() < 2e-5


def test_forward_invariants_gpu():
    _say("forward invariants")
    sc = scenes.tiny_scene(seed=4)
    _, got, pr, _ = _forward_case(sc)
    assert got["t_final"].min() >= np.float32(1e-4)
    assert got["rgb"].min() >= 0 and got["rgb"].max() <= 1 + 1e-6
    assert np.array_equal(got["n_contrib"] == 0, got["sil"] == 0)


# ---------------------------------------------------------------- backward

def _grad_maps(rng, H, W, C):
    return {"rgb": rng.standard_normal((H, W, 3)).astype(np.float32),
            "depth": rng.standard_normal((H, W)).astype(np.float32),
            "sil": rng.standard_normal((H, W)).astype(np.float32),
            "sem": rng.standard_normal((H, W, C)).astype(np.float32)}


def _backward_case(sc, semgeo, seed=0):
    cam = sc.cameras[0]
    rng = np.random.default_rng(seed)
    dl = _grad_maps(rng, cam.height, cam.width, sc.num_classes)
    fr = U.frame_for(sc, semgeo=semgeo)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    gg = {k: torch.from_numpy(v).cuda().reshape(cam.height * cam.width, -1).squeeze(-1).contiguous()
          for k, v in dl.items()}
    maps = fr.forward(g)
    out = fr.backward(g, gg)
    torch.cuda.synchronize()
    got = {k: U.to_np(v) for k, v in out.items()}
    view = U.OracleView.of_scene(sc, cfg=U.oracle_cfg(semgeo=semgeo))
    mrep = U.compare_maps({k: fr.split(v)[0].cpu().numpy() for k, v in maps.items()}, view)
    want = view.backward(dl)
    grep = U.compare_grads(got, want, view.excluded(), visible=view.pr["visible"])
    return {"maps": mrep, "grads": grep}


@pytest.mark.parametrize("semgeo", [0, 1])
def test_backward_tiny(semgeo):
    _say("backward tiny", semgeo)
    sc = scenes.tiny_scene(seed=5)
    # anisotropic, rotated Gaussians so every chain-rule term is exercised
    rng = np.random.default_rng(9)
    sc.scales = (sc.scales * np.exp(rng.normal(0, 0.4, sc.scales.shape))).astype(np.float32)
    q = rng.standard_normal((sc.n, 4))
    sc.quats = (q / np.linalg.norm(q, axis=1, keepdims=True) * 1.7).astype(np.float32)
    _backward_case(sc, semgeo)


def test_backward_room_full_frame():
    _say("backward room 200k 1200x680")
    sc = _room_crop()
    rep = _backward_case(sc, 0)
    print("backward room report", rep, flush=True)


def test_autograd_matches_frame_backward():
    _say("autograd")
    sc = scenes.tiny_scene(seed=6)
    g = Gaussians.from_scene(sc)
    params = [g.means, g.scales, g.quats, g.opacity, g.rgb, g.sem_val]
    for p in params:
        p.requires_grad_(True)
    fr = U.frame_for(sc)
    out = render(g, fr)
    rng = np.random.default_rng(1)
    w = {k: torch.from_numpy(rng.standard_normal(tuple(out[k].shape)).astype(np.float32)).cuda()
         for k in ("rgb", "depth", "sil", "sem")}
    loss = sum((out[k] * w[k]).sum() for k in w)
    loss.backward()
    g2 = Gaussians(*[p.detach() for p in params], g.sem_idx)
    fr2 = U.frame_for(sc)
    fr2.prepare(g2)
    fr2.forward(g2)
    ref = fr2.backward(g2, dict(w))
    for name, p in zip(("means", "scales", "quats", "opacity", "rgb", "sem_val"), params):
        assert torch.equal(p.grad, ref[name]), name


def test_render_backward_after_another_call_raises():
    """The autograd backward reads what its forward left in the frame's
    workspace: after another render on the same frame it raises instead of
    returning the other render's gradients, and an in-place update of a
    parameter between forward and backward is rejected by autograd."""
    _say("stale backward")
    sc = scenes.tiny_scene(seed=6)
    g = Gaussians.from_scene(sc)
    for p in (g.means, g.scales, g.quats, g.opacity, g.rgb, g.sem_val):
        p.requires_grad_(True)
    fr = U.frame_for(sc)
    first = render(g, fr)
    second = render(g, fr)
    with pytest.raises(RuntimeError, match="frame was used"):
        first["rgb"].sum().backward()
    second["rgb"].sum().backward()  # the latest render still differentiates
    assert g.means.grad is not None
    fr2 = U.frame_for(sc)
    out = render(g, fr2)
    with torch.no_grad():
        g.opacity.mul_(0.5)
    with pytest.raises(RuntimeError):
        out["sil"].sum().backward()
    torch.cuda.synchronize()


# ---------------------------------------------------------------- determinism and edge cases

def test_bitwise_determinism():
    _say("determinism")
    sc = scenes.tiny_scene(seed=7)
    g = Gaussians.from_scene(sc)
    res = []
    for _ in range(2):
        fr = U.frame_for(sc)
        fr.prepare(g)
        maps = fr.forward(g)
        dl = {k: torch.ones_like(maps[k]) for k in ("rgb", "depth", "sil", "sem")}
        grads = fr.backward(g, dl)
        torch.cuda.synchronize()
        res.append(({k: v.clone() for k, v in maps.items()}, {k: v.clone() for k, v in grads.items()}))
    for k in res[0][0]:
        assert torch.equal(res[0][0][k], res[1][0][k]), k
    for k in res[0][1]:
        assert torch.equal(res[0][1][k], res[1][1][k]), k


def test_backward_halves_equal_full_backward():
    """sgr_render_backward_tiles followed by sgr_render_backward_gather gives
    the bits of sgr_render_backward."""
    _say("backward halves")
    sc = scenes.tiny_scene(seed=9)
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    fr.prepare(g)
    maps = fr.forward(g)
    gen = torch.Generator(device="cuda").manual_seed(3)
    dl = {k: torch.randn(maps[k].shape, generator=gen, device="cuda") for k in ("rgb", "depth", "sil", "sem")}
    full = {k: v.clone() for k, v in fr.backward(g, dict(dl)).items()}
    fr.backward_tiles(g, dict(dl))
    halves = fr.backward_gather(g)
    torch.cuda.synchronize()
    for k in full:
        assert torch.equal(full[k], halves[k]), k


def test_permutation_invariance():
    _say("permutation")
    sc = scenes.tiny_scene(seed=8)
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, sc.cameras[0], O.config_array())
    zb = pr["zbits"][pr["visible"] == 1]
    assert len(np.unique(zb)) == len(zb), "depth ties: pick another seed"
    perm = np.random.default_rng(0).permutation(sc.n)
    sc2 = scenes.Scene(sc.means[perm], sc.scales[perm], sc.quats[perm], sc.opacity[perm], sc.rgb[perm],
                       sc.sem_val[perm], sc.sem_idx[perm], sc.num_classes, sc.cameras)
    outs = []
    for s in (sc, sc2):
        fr = U.frame_for(s)
        g = Gaussians.from_scene(s)
        fr.prepare(g)
        outs.append(fr.forward(g))
    torch.cuda.synchronize()
    for k in outs[0]:
        assert torch.equal(outs[0][k], outs[1][k]), k


def test_capacity_overflow_reported_and_recovered():
    _say("capacity")
    sc = scenes.tiny_scene(seed=0)
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, sc.cameras[0], O.config_array())
    K = len(O.reference_keys([pr], sc.cameras)[0])
    fr = U.frame_for(sc, cap=K - 1)
    g = Gaussians.from_scene(sc)
    fr.project(g)
    fr.bin(g)
    st, nv, nk = fr.status()
    assert st == 2 and nk == K and nv == int(pr["visible"].sum())
    maps = fr.forward(g)  # does no work on an overflowed frame, and must not fault
    torch.cuda.synchronize()
    fr.prepare(g)  # grows the capacity
    st, _, nk = fr.status()
    assert st == 0 and nk == K and fr.key_capacity >= K


def test_empty_and_fully_culled_scenes():
    _say("empty")
    sc = scenes.tiny_scene(seed=0, n=64)
    sc.means[:, 2] = -5.0  # everything behind the camera
    fr = U.frame_for(sc)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    maps = fr.forward(g)
    ne, hs = fr.score(g)
    torch.cuda.synchronize()
    assert torch.all(maps["t_final"] == 1) and torch.all(maps["n_contrib"] == 0)
    assert torch.all(maps["rgb"] == 0) and torch.all(maps["sem"] == 0)
    P = 64 * 64
    assert int(ne[0]) == P
    assert math.isclose(float(hs[0]), P * math.log(sc.num_classes), rel_tol=1e-6)
    sc0 = scenes.tiny_scene(seed=0, n=0)
    fr0 = U.frame_for(sc0)
    g0 = Gaussians.from_scene(sc0)
    fr0.prepare(g0)
    maps0 = fr0.forward(g0)
    torch.cuda.synchronize()
    assert torch.all(maps0["t_final"] == 1)


# ---------------------------------------------------------------- scoring

def test_score_views_vs_oracle_and_plain_path():
    _say("score views")
    sc = scenes.candidate_scene(n=60_000, nviews=6)
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    ne, hs = fr.score(g)
    st, _, _ = fr.status()
    assert st == 0
    ne, hs = U.to_np(ne).astype(np.int64), U.to_np(hs)
    cfg = U.oracle_cfg()
    for v, cam in enumerate(sc.cameras):
        pr, mp = O.forward(O.scene_arrays(sc), cam, cfg, sc.num_classes)
        sref = O.score(mp, sc.num_classes)
        P = cam.width * cam.height
        slack = int(((mp["flags"] != 0) & (mp["n_contrib"] <= 1)).sum())
        assert abs(int(ne[v]) - sref["n_empty"]) <= slack, (v, ne[v], sref["n_empty"])
        assert abs(hs[v] - sref["entropy_sum"]) / P <= 1e-4, (v, hs[v], sref["entropy_sum"])
        # plain one-view path: project, bin, dense render, separate reduction
        f1 = U.frame_for(sc, cams=[cam])
        f1.prepare(g)
        maps = f1.forward(g, f1.alloc_maps(want=("sem",)))
        pe, ph = score_maps(maps["sem"].reshape(cam.height, cam.width, -1),
                            maps["n_contrib"].reshape(cam.height, cam.width), sc.num_classes)
        torch.cuda.synchronize()
        assert int(pe[0]) == int(ne[v])
        assert abs(float(ph[0]) - hs[v]) <= 1e-9 * P


@pytest.mark.parametrize("acc", [1, 2])
def test_duplicate_top_k_classes_add(acc):
    """Repeated class indices within a Gaussian's top-k add (Eq. 3 with
    p_{i,m} the sum of its entries); checked against the oracle with the
    class sums in LDS (1) and in registers (2)."""
    _say("duplicate classes", acc)
    sc = scenes.tiny_scene(seed=9)
    rng = np.random.default_rng(3)
    dup = rng.random(sc.n) < 0.3
    sc.sem_idx[dup, 1] = sc.sem_idx[dup, 0]
    fr = U.frame_for(sc, acc=acc)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    maps = fr.forward(g)
    torch.cuda.synchronize()
    got = {k: fr.split(v)[0].cpu().numpy() for k, v in maps.items()}
    rep = U.compare_maps(got, U.OracleView.of_scene(sc))
    assert rep["unresolved"] == 0, rep


@pytest.mark.parametrize("case", ["tiny_c16", "room_c102", "tiny_c110"])
def test_accumulator_placements_give_identical_bits(case):
    """Class sums in LDS and in registers (the autotuner's choice) give the
    same bits for maps, gradients and scores (C = 110 fills the fourth
    register vector almost to the end)."""
    _say("accumulators", case)
    if case == "tiny_c16":
        sc = scenes.tiny_scene(seed=11)
    elif case == "tiny_c110":
        sc = scenes.tiny_scene(seed=12, num_classes=110, k=16)
    else:
        sc = _room_crop(n=60_000, w=400, h=300)
    g = Gaussians.from_scene(sc)
    cam = sc.cameras[0]
    P = cam.width * cam.height
    rng = np.random.default_rng(5)
    dl = {k: torch.from_numpy(v).cuda().reshape(P, -1).squeeze(-1).contiguous()
          for k, v in _grad_maps(rng, cam.height, cam.width, sc.num_classes).items()}
    modes = [0, 1, 2]
    res = []
    for acc in modes:
        fr = U.frame_for(sc, acc=acc)
        fr.prepare(g)
        maps = {k: v.clone() for k, v in fr.forward(g).items()}
        grads = {k: v.clone() for k, v in fr.backward(g, dict(dl)).items()}
        ne, hs = fr.score(g)
        torch.cuda.synchronize()
        res.append((maps, grads, ne.clone(), hs.clone()))
    for other in res[1:]:
        for k in res[0][0]:
            assert torch.equal(res[0][0][k], other[0][k]), k
        for k in res[0][1]:
            assert torch.equal(res[0][1][k], other[1][k]), k
        assert torch.equal(res[0][2], other[2]) and torch.equal(res[0][3], other[3])


@pytest.mark.parametrize("case", ["tiny_c16", "room_c102", "tiny_c256"])
def test_class_passes_give_identical_bits(case):
    """Class sums split into 2..4 ranges composited one after another give
    the bits of a single pass: maps, scores and the fused cross-entropy loss
    with its gradients.  At C = 256 a single pass does not fit the LDS: the
    forward then accumulates in the output map (same bits), while scoring
    and the fused loss asked for the semantic map report SGR_EUNSUPPORTED."""
    _say("class passes", case)
    if case == "tiny_c16":
        sc = scenes.tiny_scene(seed=14)
    elif case == "tiny_c256":
        sc = scenes.tiny_scene(seed=15, num_classes=256, k=16)
    else:
        sc = _room_crop(n=60_000, w=400, h=300)
    g = Gaussians.from_scene(sc)
    cam = sc.cameras[0]
    P, C = cam.width * cam.height, sc.num_classes
    rng = np.random.default_rng(6)
    tg = {"rgb": torch.from_numpy(rng.random((P, 3)).astype(np.float32)),
          "depth": torch.from_numpy((rng.random(P) * 4.5 + 0.5).astype(np.float32)),
          "label": torch.from_numpy(rng.integers(0, C, size=P).astype(np.int32))}
    fwd, rest = [], []
    for passes in (1, 2, 3, 4):
        fr = U.frame_for(sc, passes=passes)
        fr.prepare(g)
        fwd.append({k: v.clone() for k, v in fr.forward(g).items()})
        if case == "tiny_c256" and passes == 1:
            with pytest.raises(SgrError):
                fr.score(g)
            with pytest.raises(SgrError):
                fr.forward_loss(g, tg, maps=fr.alloc_maps(), sparse_sem=True)
            continue
        ne, hs = fr.score(g)
        maps = fr.alloc_maps()
        gr, loss = fr.forward_loss(g, tg, maps=maps, sparse_sem=True)
        torch.cuda.synchronize()
        rest.append((ne.clone(), hs.clone(), {k: v.clone() for k, v in gr.items()}, loss.clone(), maps))
    torch.cuda.synchronize()
    for other in fwd[1:]:
        for k in fwd[0]:
            assert torch.equal(fwd[0][k], other[k]), k
    for ne, hs, gr, loss, maps in rest[1:]:
        assert torch.equal(rest[0][0], ne) and torch.equal(rest[0][1], hs)
        assert torch.equal(rest[0][3], loss)
        for k in gr:
            assert torch.equal(rest[0][2][k], gr[k]), k
        for k in maps:
            assert torch.equal(rest[0][4][k], maps[k]), k
    for k in rest[0][4]:  # the fused launch writes the forward's maps
        assert torch.equal(rest[0][4][k], fwd[-1][k]), k


def test_out_of_range_class_index_reported():
    """An index >= C is an input error: reported as SGR_EINVAL by the status
    word, never used to address memory."""
    _say("bad class index")
    sc = scenes.tiny_scene(seed=10)
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, sc.cameras[0], O.config_array())
    i = int(np.nonzero(pr["visible"])[0][0])
    sc.sem_idx[i, 0] = sc.num_classes + 3
    fr = U.frame_for(sc)
    g = Gaussians.from_scene(sc)
    with pytest.raises(Exception) as e:
        fr.prepare(g)
    assert getattr(e.value, "status", None) == 1
    fr.forward(g)
    torch.cuda.synchronize()


def test_multiview_forward_backward_sums_over_views():
    """Three keyframes rendered and differentiated in one batch; the
    gradient is the sum of the per-view oracle gradients."""
    _say("multiview fwd+bwd")
    sc = scenes.room_scene(n=30_000, targets=False)
    base = sc.cameras[0]
    cams = []
    for j, (w, h) in enumerate([(320, 200), (256, 256), (400, 150)]):
        c = scenes.look_at(base.center + np.array([0.3 * j, -0.2 * j, 0.1 * j]),
                           base.center + np.array([3.0, 0.5 * (j - 1), 0.0]), w, h, 0.6 * w, 0.6 * w)
        cams.append(c)
    sc.cameras = cams
    rng = np.random.default_rng(4)
    fr = U.frame_for(sc)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    maps = fr.forward(g)
    dls = [_grad_maps(rng, c.height, c.width, sc.num_classes) for c in cams]
    flat = {k: torch.from_numpy(np.concatenate([d[k].reshape(c.height * c.width, -1) for d, c in zip(dls, cams)])
                                ).cuda().squeeze(-1).contiguous() for k in ("rgb", "depth", "sil", "sem")}
    out = fr.backward(g, flat)
    torch.cuda.synchronize()
    got = {k: U.to_np(v) for k, v in out.items()}
    cfg = U.oracle_cfg()
    want, bad, vis = None, np.zeros(sc.n, bool), np.zeros(sc.n, bool)
    for v, (c, dl) in enumerate(zip(cams, dls)):
        view = U.OracleView.of_scene(sc, cam=c, cfg=cfg)
        U.compare_maps({k: fr.split(maps[k])[v].cpu().numpy() for k in maps}, view)
        gv = view.backward(dl)
        want = gv if want is None else {k: want[k] + gv[k] for k in want}
        bad |= view.excluded()
        vis |= view.pr["visible"] == 1
    print("multiview report", U.compare_grads(got, want, bad, visible=vis), flush=True)


def test_full_size_mapping_frame_1m():
    """The benchmarked workload at full size: 1M Gaussians, 1200x680, with
    the key capacity and launch configuration the benchmark uses; forward
    maps and gradients against the oracle."""
    _say("full size 1M 1200x680")
    sc = scenes.room_scene(n=1_000_000, targets=False)
    cam = sc.cameras[0]
    fr = U.frame_for(sc)
    g = Gaussians.from_scene(sc)
    fr.prepare(g)
    _, _, nk = fr.status()
    fr.key_capacity = int(nk * 1.5) + 4096
    fr._alloc()
    fr.prepare(g, check=False)
    maps = fr.forward(g)
    st, _, _ = fr.status()
    assert st == 0
    rng = np.random.default_rng(11)
    dl = _grad_maps(rng, cam.height, cam.width, sc.num_classes)
    gg = {k: torch.from_numpy(v).cuda().reshape(cam.height * cam.width, -1).squeeze(-1).contiguous()
          for k, v in dl.items()}
    out = fr.backward(g, gg)
    torch.cuda.synchronize()
    got_maps = {k: fr.split(v)[0].cpu().numpy() for k, v in maps.items()}
    view = U.OracleView.of_scene(sc)
    rep = U.compare_maps(got_maps, view)
    assert rep["flagged"] <= 0.002 * view.flags.size, rep
    want = view.backward(dl)
    got = {k: U.to_np(v) for k, v in out.items()}
    print("full size report", rep, U.compare_grads(got, want, view.excluded(), visible=view.pr["visible"]),
          flush=True)


def test_score_views_graph_replay_matches_eager():
    """sgr_score_views captured in a HIP graph: every replay, with eager work
    and synchronisations in between, equals the eager result bit for bit."""
    _say("score graph")
    sc = scenes.candidate_scene(n=40_000, nviews=7)
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    ne0, hs0 = fr.score(g)
    torch.cuda.synchronize()
    ne0, hs0 = ne0.clone(), hs0.clone()
    graph, ne, hs = fr.capture_score(g)
    for r in range(4):
        ne.fill_(-1)
        hs.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(ne, ne0) and torch.equal(hs, hs0), r
        fr.score(g)  # eager work between replays
        torch.cuda.synchronize()
    st, _, _ = fr.status()
    assert st == 0


def test_autotuner_choices_keep_outputs(tmp_path, monkeypatch):
    """The autotuner times every candidate on the frame's own data, checks
    that all candidates give the same bits, and leaves the fastest in the
    config (also in its JSON cache, keyed by architecture and shape); the
    tuned frame reproduces the default frame's outputs."""
    _say("autotune")
    monkeypatch.setenv("SGR_AUTOTUNE_CACHE", str(tmp_path / "autotune.json"))
    autotune.clear_cache()
    sc = scenes.candidate_scene(n=30_000, nviews=4)
    g = Gaussians.from_scene(sc)
    fr = U.frame_for(sc)
    fr.prepare(g)
    rep = autotune.tune_mapping(fr, g, reps=1)
    # stage one: placements (LDS in 1, 2 or 3 class ranges, registers) x two
    # tile orders; stage two: three backward batches x two digit widths
    assert len(rep["candidates"]) == 8 + 6 and rep["chosen"] in rep["candidates"]
    rep2 = autotune.tune_score(fr, g, reps=1, workgroups=(0, 64))
    assert len(rep2["candidates"]) == 16 + 2
    knobs = {k: int(getattr(fr.cfg, k)) for k in autotune.KNOBS}
    assert autotune.tune_score(fr, g)["cached"] == knobs
    autotune.clear_cache()  # the JSON file still has it
    assert autotune.tune_score(fr, g)["cached"] == knobs
    rng = np.random.default_rng(2)
    tg = [{"rgb": torch.from_numpy(rng.random((c.width * c.height, 3)).astype(np.float32)),
           "depth": torch.from_numpy(rng.random(c.width * c.height).astype(np.float32) + 1.0),
           "label": torch.from_numpy(rng.integers(0, sc.num_classes, c.width * c.height).astype(np.int32))}
          for c in sc.cameras]
    rep3 = autotune.tune_mapping(fr, g, reps=1, targets=tg)
    assert rep3["what"] == "mapping_loss" and len(rep3["candidates"]) == 8 + 6
    ref = U.frame_for(sc)
    ref.prepare(g)
    fr.prepare(g)
    a, b = ref.forward(g), fr.forward(g)
    sa, sb = ref.score(g), fr.score(g)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(sa[0], sb[0]) and torch.equal(sa[1], sb[1])
