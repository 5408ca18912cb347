"""The benchmarked mapping step at full size, stage by stage, against the
FP64 oracle; and two portrait keyframes of the large multi-room workload
rendered and differentiated in one batch.

The mapping step runs exactly the launches the benchmark times: the fused
forward with the mapping loss and label-only class sums (cross-entropy,
its gradient kept as one class per pixel), the backward over the tiles with
that one-class gradient, and the gather with the chain rule to 3D.  Each
stage meets the oracle (Eq. 1 / Eq. 3 forward, the Sec. 3.1 loss, the
analytic backward), flagged pixels on the outcome the GPU took:

* maps of the same launch: 1e-4 absolute, n_contrib exact;
* loss: 1e-5 relative to the loss oracle on the oracle's maps;
* dL/dmaps: element-wise against the loss oracle on the oracle's maps;
  the cross-entropy gradient -1/(P q) is compared with the 1e-4 map bar
  carried through it (relative 1e-3 + 1e-4 / q);
* parameter gradients: the oracle's backward fed with the GPU's dL/dmaps,
  all six tensors element-wise to 1e-3 on at least 99 % of the visible
  Gaussians, and the whole oracle chain (oracle maps -> loss oracle ->
  oracle backward) to 1e-3 in relative L2.
"""
import numpy as np
import pytest
import torch

from oracle import loss as OL
from paper_2506_00225_amd import Frame, Gaussians, loss_config, make_config, scenes

import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00225_amd import _lib
    _lib.lib()


def _say(*a):
    print("[case]", *a, flush=True)


def _bench_frame(sc, cams):
    """A frame sized as the benchmark sizes it: key capacity 1.5x the
    measured key count."""
    g = Gaussians.from_scene(sc)
    fr = Frame(sc.n, cams, make_config(sc.num_classes, sc.k))
    fr.prepare(g)
    _, _, nk = fr.status()
    fr.key_capacity = int(nk * 1.5) + 4096
    fr._alloc()
    fr.prepare(g)
    return g, fr


def test_benchmarked_mapping_step_1m():
    _say("benchmarked mapping step 1M 1200x680")
    sc = scenes.room_scene(n=1_000_000)
    cam = sc.cameras[0]
    H, W, C, k = cam.height, cam.width, sc.num_classes, sc.k
    P = H * W
    g, fr = _bench_frame(sc, [cam])
    dev = g.means.device
    label = torch.from_numpy(sc.targets["label"]).to(dev).reshape(P).int().contiguous()
    targets = {"rgb": torch.from_numpy(sc.targets["rgb"]).to(dev).reshape(P, 3),
               "depth": torch.from_numpy(sc.targets["depth"]).to(dev).reshape(P), "label": label}
    grads_in = {"rgb": torch.empty(P, 3, device=dev), "depth": torch.empty(P, device=dev),
                "sil": torch.empty(P, device=dev), "sem_at_label": torch.empty(P, device=dev), "sem_label": label}
    maps = {"rgb": torch.empty(P, 3, device=dev), "depth": torch.empty(P, device=dev),
            "sil": torch.empty(P, device=dev), "t_final": torch.empty(P, device=dev),
            "n_contrib": torch.empty(P, dtype=torch.int32, device=dev)}
    gout = {nm: torch.empty_like(getattr(g, nm)) for nm in ("means", "scales", "quats", "opacity", "rgb", "sem_val")}
    _, loss = fr.forward_loss(g, targets, loss_config(), maps=maps, grads=grads_in)
    fr.backward_tiles(g, grads_in)
    fr.backward_gather(g, gout)
    torch.cuda.synchronize()
    assert fr.status()[0] == 0

    # forward maps of the same launch
    view = U.OracleView.of_scene(sc)
    got_maps = {kk: U.to_np(v).reshape((H, W, 3) if kk == "rgb" else (H, W)) for kk, v in maps.items()}
    mrep = U.compare_maps(got_maps, view)
    assert mrep["flagged"] <= 0.002 * P and mrep["unresolved"] == 0, mrep
    om = view.maps()

    # the loss and its gradient with respect to the maps
    t = {"rgb": sc.targets["rgb"], "depth": sc.targets["depth"], "label": sc.targets["label"]}
    want_loss, wg, lflags = OL.mapping_loss(om, t, C, k)
    assert float(loss[0]) == pytest.approx(want_loss, rel=1e-5)
    ok = ~lflags
    for key, shape in (("rgb", (H, W, 3)), ("depth", (H, W)), ("sil", (H, W))):
        gv = U.to_np(grads_in[key]).reshape(shape).astype(np.float64)
        scale = np.abs(wg[key]).max() + 1e-30
        assert np.allclose(gv[ok], wg[key][ok], rtol=1e-3, atol=1e-5 * scale), key
    lab = sc.targets["label"].astype(np.int64)
    q = np.take_along_axis(om["sem"], lab[..., None], -1)[..., 0]
    want_gl = np.take_along_axis(wg["sem"], lab[..., None], -1)[..., 0]
    gl = U.to_np(grads_in["sem_at_label"]).reshape(H, W).astype(np.float64)
    tol = (1e-3 + 1e-4 / np.maximum(q, 1e-6)) * np.abs(want_gl) + 1e-12
    bad = (np.abs(gl - want_gl) > tol) & ok
    assert not bad.any(), (int(bad.sum()), float(np.abs(gl - want_gl)[bad].max()))

    # parameter gradients: the oracle's backward fed with the GPU's dL/dmaps ...
    got = {kk: U.to_np(v) for kk, v in gout.items()}
    dense = np.zeros((H, W, C))
    np.put_along_axis(dense, lab[..., None], gl[..., None], -1)
    dl_gpu = {"rgb": U.to_np(grads_in["rgb"]).reshape(H, W, 3), "depth": U.to_np(grads_in["depth"]).reshape(H, W),
              "sil": U.to_np(grads_in["sil"]).reshape(H, W), "sem": dense}
    grep = U.compare_grads(got, view.backward(dl_gpu), view.excluded(), visible=view.pr["visible"])
    # ... and the whole oracle chain, in relative L2
    chain = view.backward(wg)
    l2 = {kk: float(np.linalg.norm(got[kk] - chain[kk]) / (np.linalg.norm(chain[kk]) + 1e-30)) for kk in chain}
    print("mapping step report", mrep, grep, "chain L2", l2, flush=True)
    for kk, e in l2.items():
        assert e <= 1e-3, (kk, l2)


def test_large_scene_two_portrait_keyframes():
    """Two 1024x1280 keyframes of the 3M-Gaussian multi-room scene (C = 40)
    in one batch, forward and backward: each view's maps against the oracle
    and the gradients against the sum of the per-view oracle gradients,
    element-wise on every visible Gaussian (Gaussians near the camera cover
    up to the whole 1.3M-pixel view, thin ones have conics of condition
    number in the thousands)."""
    _say("large scene 3M, 2 x 1024x1280, C=40")
    sc = scenes.large_scene()
    cams = sc.cameras[:2]
    g, fr = _bench_frame(sc, cams)
    maps = fr.forward(g)
    rng = np.random.default_rng(17)
    C = sc.num_classes
    dls = [{"rgb": rng.standard_normal((c.height, c.width, 3)).astype(np.float32),
            "depth": rng.standard_normal((c.height, c.width)).astype(np.float32),
            "sil": rng.standard_normal((c.height, c.width)).astype(np.float32),
            "sem": rng.standard_normal((c.height, c.width, C)).astype(np.float32)} for c in cams]
    flat = {kk: torch.from_numpy(np.concatenate([d[kk].reshape(c.height * c.width, -1) for d, c in zip(dls, cams)])
                                 ).cuda().squeeze(-1).contiguous() for kk in ("rgb", "depth", "sil", "sem")}
    out = fr.backward(g, flat)
    torch.cuda.synchronize()
    assert fr.status()[0] == 0
    got = {kk: U.to_np(v) for kk, v in out.items()}
    want, bad, vis = None, np.zeros(sc.n, bool), np.zeros(sc.n, bool)
    reps = []
    for v, (c, dl) in enumerate(zip(cams, dls)):
        view = U.OracleView.of_scene(sc, cam=c)
        rep = U.compare_maps({kk: fr.split(maps[kk])[v].cpu().numpy() for kk in maps}, view)
        assert rep["unresolved"] == 0, rep
        reps.append(rep)
        gv = view.backward(dl)
        want = gv if want is None else {kk: want[kk] + gv[kk] for kk in want}
        bad |= view.excluded()
        vis |= view.pr["visible"] == 1
    print("large scene report", reps, U.compare_grads(got, want, bad, visible=vis), flush=True)


@pytest.mark.parametrize("n,k", [(200_000, 16), (60_000, 3), (60_000, 5)])
def test_gather_with_adam_equals_gather_then_adam(n, k):
    """The gather with the Adam step fused (sgr_render_backward_gather_adam)
    gives, bit for bit, the parameters and moments of the gather followed by
    sgr_adam_step, over two mapping iterations of a room (the second starts
    from nonzero moments): top-16 lists, and the kernels for 3 entries and
    for a run-time list length."""
    from paper_2506_00225_amd import FusedAdam
    _say(f"gather + Adam fused vs separate, {n} Gaussians, k={k}")
    sc = scenes.room_scene(n=n, k=k)
    cam = sc.cameras[0]
    P = cam.width * cam.height
    g0, fr = _bench_frame(sc, [cam])
    dev = g0.means.device
    label = torch.from_numpy(sc.targets["label"]).to(dev).reshape(P).int().contiguous()
    targets = {"rgb": torch.from_numpy(sc.targets["rgb"]).to(dev).reshape(P, 3),
               "depth": torch.from_numpy(sc.targets["depth"]).to(dev).reshape(P), "label": label}
    names = ("means", "scales", "quats", "opacity", "rgb", "sem_val")
    inf = float("inf")
    clamp = {"opacity": (1e-4, 0.9999), "sem_val": (0.0, inf)}
    runs = []
    for fused in (False, True):
        g = Gaussians(*[getattr(g0, nm).clone() for nm in names], g0.sem_idx)
        gout = {nm: torch.empty_like(getattr(g, nm)) for nm in names}
        opt = FusedAdam([(getattr(g, nm), gout[nm], *clamp.get(nm, (-inf, inf))) for nm in names], lr=1e-3)
        grads_in = {"rgb": torch.empty(P, 3, device=dev), "depth": torch.empty(P, device=dev),
                    "sil": torch.empty(P, device=dev), "sem_at_label": torch.empty(P, device=dev),
                    "sem_label": label}
        for _ in range(2):
            fr.project(g)
            fr.bin(g)
            fr.forward_loss(g, targets, loss_config(), grads=grads_in)
            fr.backward_tiles(g, grads_in)
            if fused:
                fr.backward_gather_adam(g, opt)
            else:
                fr.backward_gather(g, gout)
                opt.step()
        torch.cuda.synchronize()
        assert fr.status()[0] == 0
        runs.append(([getattr(g, nm).clone() for nm in names], [m.clone() for m in opt.m], [v.clone() for v in opt.v]))
    (pa, ma, va), (pb, mb, vb) = runs
    for nm, x, y in zip(names, pa, pb):
        assert torch.equal(x, y), nm
    for nm, x, y in zip(names + names, ma + va, mb + vb):
        assert torch.equal(x, y), nm
    assert not torch.equal(pa[0], g0.means)  # the step did move the means
