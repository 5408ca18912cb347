"""Top-k semantic state kernels (selection at initialisation, fixed-index
updates) against the oracle, and a render of freshly selected state."""
import numpy as np
import pytest
import torch

from oracle import topk as OT
from paper_2506_00225_amd import Gaussians, scenes, topk_select, topk_update

import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("k", [3, 16, 20])
@pytest.mark.parametrize("renorm", [False, True])
def test_topk_select_matches_oracle(k, renorm):
    print("[case] topk select", k, renorm, flush=True)
    rng = np.random.default_rng(k)
    rows, C = 3000, 102
    dist = (np.round(rng.random((rows, C)) * 16) / 16).astype(np.float32)  # many equal values
    dist[rng.random((rows, C)) < 0.01] = np.nan
    pixel = rng.integers(0, rows, size=5000)
    idx, val = topk_select(torch.from_numpy(dist).cuda(), k, torch.from_numpy(pixel).cuda(), renormalize=renorm)
    torch.cuda.synchronize()
    widx, wval = OT.select(dist, pixel, k, renormalize=renorm)
    assert np.array_equal(U.to_np(idx), widx)
    assert np.array_equal(U.to_np(val), wval)


def test_topk_update_matches_oracle():
    print("[case] topk update", flush=True)
    rng = np.random.default_rng(1)
    dist = rng.random((400, 40)).astype(np.float32)
    idx, val = OT.select(dist, None, 16)
    pixel = rng.integers(0, 400, size=400)
    g_idx, g_val = torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda()
    topk_update(torch.from_numpy(dist).cuda(), g_idx, g_val, 0.3, torch.from_numpy(pixel).cuda())
    torch.cuda.synchronize()
    want = OT.update(dist, pixel, idx, val, 0.3)
    assert np.allclose(U.to_np(g_val), want, rtol=0, atol=1e-7)


def test_selected_state_renders_like_its_dense_rows():
    """Gaussians initialised by top-k selection from dense distributions
    render (top-k forward) exactly like the dense forward of those rows with
    every class outside the top-k zeroed."""
    print("[case] topk render", flush=True)
    sc = scenes.tiny_scene(seed=21, num_classes=40, k=8)
    rng = np.random.default_rng(2)
    dense = rng.dirichlet(np.ones(40) * 0.3, size=sc.n).astype(np.float32)
    idx, val = topk_select(torch.from_numpy(dense).cuda(), 8)
    g = Gaussians.from_scene(sc)
    g.sem_idx, g.sem_val = idx, val
    fr = U.frame_for(sc)
    fr.prepare(g)
    a = {k: v.clone() for k, v in fr.forward(g).items()}
    kept = np.zeros_like(dense)
    np.put_along_axis(kept, U.to_np(idx).astype(np.int64), U.to_np(val), axis=1)
    b = fr.forward_dense(g, torch.from_numpy(kept))
    torch.cuda.synchronize()
    for key in a:
        assert torch.equal(a[key], b[key]), key
