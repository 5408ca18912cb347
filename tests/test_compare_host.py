"""The GPU parity helpers' handling of flagged pixels, on the CPU: maps
taken from arbitrary outcomes of the flagged decisions (rounded to float32,
as a GPU would return them) are explained branch by branch, and a value no
outcome explains is caught."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_00225_amd import scenes

import gpu_util as U


def _fake_gpu(view, branch):
    _, _, _, opacity, rgb, sem_val, sem_idx = view.arrays
    mp = O.render(view.pr, opacity, rgb, sem_val, sem_idx, view.C, view.cam, view.cfg, branch=branch)
    got = {k: mp[k].astype(np.float32) for k in ("rgb", "depth", "sil", "sem", "t_final")}
    got["n_contrib"] = mp["n_contrib"].copy()
    return got


def _view(seed=3):
    sc = scenes.tiny_scene(seed=seed, n=800, width=32, height=24, f=24.0)
    cfg = O.config_array(margin_alpha=0.05, margin_t=0.3)  # wide margins: many flagged pixels
    return sc, U.OracleView(O.scene_arrays(sc), sc.cameras[0], cfg, sc.num_classes)


def test_resolve_explains_any_outcome():
    sc, view = _view()
    flagged = view.flags != 0
    assert flagged.sum() > 40
    rng = np.random.default_rng(0)
    branch = np.where(flagged, rng.integers(0, 16, size=flagged.shape), 0).astype(np.uint32)
    got = _fake_gpu(view, branch)
    rep = U.compare_maps(got, view, atol=1e-5)
    assert rep["unresolved"] == 0 and rep["non_default"] > 10, rep
    want = view.maps()
    for key in ("rgb", "sil", "sem", "t_final"):
        assert np.abs(want[key] - got[key]).max() < 1e-6, key
    assert np.array_equal(want["n_contrib"], got["n_contrib"])


def test_resolve_rejects_a_value_no_outcome_gives():
    sc, view = _view(seed=4)
    got = _fake_gpu(view, np.zeros_like(view.branch))
    ys, xs = np.nonzero(view.flags)
    got["rgb"][ys[0], xs[0], 1] += 0.05  # planted in the stand-in for the GPU result
    with pytest.raises(AssertionError):
        U.compare_maps(got, view, atol=1e-5)


def test_gradients_follow_the_resolved_branches():
    """The oracle gradient on the resolved branches equals the gradient of
    the outcome the maps came from."""
    sc, view = _view(seed=5)
    flagged = view.flags != 0
    branch = np.where(flagged, 1, 0).astype(np.uint32)
    got = _fake_gpu(view, branch)
    U.compare_maps(got, view, atol=1e-5)
    cam = sc.cameras[0]
    rng = np.random.default_rng(1)
    dl = {"rgb": rng.standard_normal((cam.height, cam.width, 3)), "depth": rng.standard_normal((cam.height, cam.width)),
          "sil": rng.standard_normal((cam.height, cam.width)),
          "sem": rng.standard_normal((cam.height, cam.width, sc.num_classes))}
    a = view.backward(dl)
    b, _ = O.backward(view.arrays, cam, view.cfg, sc.num_classes, dl, proj=view.pr, branch=branch)
    for key in a:
        assert np.allclose(a[key], b[key], rtol=1e-9, atol=1e-12), key
