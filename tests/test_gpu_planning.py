"""Next-best-view planning on the GPU (candidate generation, scoring from
device poses, Eq. 5-7 combination) against the FP64 planning oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import planning as OP
from paper_2506_00225_amd import Frame, Gaussians, make_config, scenes
from paper_2506_00225_amd.planner import COARSE, FINE, Grid, Planner, sampling

import gpu_util as U

pytestmark = pytest.mark.gpu

VOXEL = 0.25
DIMS = (40, 32, 12)  # a 10 x 8 x 3 m room


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print("[case]", *a, flush=True)


def _free(radius, centre=(5.0, 4.0, 1.5)):
    """Voxels whose centre is within `radius` of `centre` (x fastest)."""
    nx, ny, nz = DIMS
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = (np.stack([x, y, z], -1) + 0.5) * VOXEL
    return (np.linalg.norm(c - np.asarray(centre), axis=-1) <= radius).astype(np.uint8).reshape(-1)


def _stage(name):
    if name == "coarse":
        return dict(COARSE, z_min=1.5, z_max=1.5)
    return dict(FINE, z_min=0.5, z_max=2.5)


def _planner(sc, w=160, h=120):
    intr = scenes.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), w / 2, w / 2, w / 2, h / 2, w, h)
    return Planner(Grid(DIMS, VOXEL, (0.0, 0.0, 0.0)), intr, make_config(sc.num_classes, sc.k), capacity=64)


@pytest.mark.parametrize("stage", ["coarse", "fine"])
def test_candidates_match_oracle(stage):
    _say("candidates", stage)
    st = _stage(stage)
    now, before = _free(4.0), _free(2.0)
    sc = scenes.tiny_scene()
    pl = _planner(sc)
    V = pl.generate(torch.from_numpy(now).cuda(), torch.from_numpy(before).cuda(),
                    sampling(st["step"], st["directions"], st["z_min"], st["z_max"]))
    poses, pos = OP.candidates(now, before, DIMS, VOXEL, (0.0, 0.0, 0.0), st["step"], st["directions"],
                               float(np.float32(st["z_min"])), float(np.float32(st["z_max"])))
    assert V == len(poses) and V > 0
    assert np.array_equal(U.to_np(pl.positions[:V]), pos)
    got = U.to_np(pl.poses[:V])
    assert np.allclose(got, poses, rtol=0, atol=2e-6)
    print("V", V, "bit-equal poses", float((got == poses).mean()), flush=True)
    # nothing new -> no candidates; nothing free before -> every lattice voxel of the ball
    assert pl.generate(torch.from_numpy(now).cuda(), torch.from_numpy(now).cuda(),
                       sampling(st["step"], st["directions"], st["z_min"], st["z_max"])) == 0
    V2 = pl.generate(torch.from_numpy(now).cuda(), None, sampling(st["step"], st["directions"], st["z_min"],
                                                                   st["z_max"]))
    assert V2 == len(OP.candidates(now, np.zeros_like(now), DIMS, VOXEL, (0.0, 0.0, 0.0), st["step"],
                                   st["directions"], float(np.float32(st["z_min"])),
                                   float(np.float32(st["z_max"])))[0])


def test_scoring_from_device_poses_and_combination():
    """sgr_score_poses gives the bits of sgr_score_views on host cameras
    built from the same poses; a subset of views is checked against the
    oracle; the combination matches the oracle's Eq. 5-7."""
    _say("score poses + combine")
    sc = scenes.room_scene(seed=3, n=40_000, targets=False)
    g = Gaussians.from_scene(sc)
    pl = _planner(sc)
    st = _stage("coarse")
    now, before = _free(4.0), _free(2.0)
    samp = sampling(st["step"], st["directions"], st["z_min"], st["z_max"])
    out = pl.step(g, torch.from_numpy(now).cuda(), torch.from_numpy(before).cuda(), samp, (5.0, 4.0, 1.5))
    V = out["V"]
    assert V > 0
    ne, hs = U.to_np(out["n_empty"]).astype(np.int64), U.to_np(out["entropy_sum"])
    poses = U.to_np(out["poses"])
    intr = pl.intr[0]
    cams = [scenes.Camera(p[:9].reshape(3, 3).copy(), p[9:].copy(), intr.fx, intr.fy, intr.cx, intr.cy, intr.width,
                          intr.height) for p in poses]
    fr = Frame(sc.n, cams, make_config(sc.num_classes, sc.k))
    ne2, hs2 = fr.score(g)
    torch.cuda.synchronize()
    assert np.array_equal(U.to_np(ne2).astype(np.int64), ne) and np.array_equal(U.to_np(hs2), hs)
    cfg = U.oracle_cfg()
    for v in range(0, V, max(1, V // 8)):
        pr, mp = O.forward(O.scene_arrays(sc), cams[v], cfg, sc.num_classes)
        ref = O.score(mp, sc.num_classes)
        slack = int(((mp["flags"] != 0) & (mp["n_contrib"] <= 1)).sum())
        assert abs(int(ne[v]) - ref["n_empty"]) <= slack
        assert abs(hs[v] - ref["entropy_sum"]) / pl.pixels <= 1e-4
    score, pruned, best = OP.combine(ne, hs, U.to_np(out["positions"]), (5.0, 4.0, 1.5), pl.pixels,
                                     prune_fraction=float(np.float32(0.005)))
    assert np.allclose(U.to_np(out["score"]), score, rtol=1e-12, atol=1e-300)
    assert np.array_equal(U.to_np(out["pruned"]).astype(bool), pruned)
    assert int(out["best"][0]) == best
    print("V", V, "pruned", int(pruned.sum()), "best", best, flush=True)


def test_combine_edge_cases():
    _say("combine edges")
    sc = scenes.tiny_scene()
    pl = _planner(sc)
    V = 5
    pl.positions[:V] = torch.tensor([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [4, 0, 0]], dtype=torch.float32)
    pl.entropy[:V] = torch.tensor([5.0, 5.0, 4.0, 1e6, 5.0], dtype=torch.float64)
    for ne in ([0, 0, 0, 0, 0], [100, 100, 50, 10, 100], [1000, 1000, 1000, 1000, 1000]):
        pl.n_empty[:V] = torch.tensor(ne, dtype=torch.int32)
        sc_, pr, best = pl.combine(V, (0.0, 0.0, 0.0), prune_fraction=0.01)
        torch.cuda.synchronize()
        s2, p2, b2 = OP.combine(np.array(ne), U.to_np(pl.entropy[:V]), U.to_np(pl.positions[:V]), (0, 0, 0),
                                pl.pixels, prune_fraction=float(np.float32(0.01)))
        assert np.allclose(U.to_np(sc_), s2, rtol=1e-12, atol=1e-300)
        assert np.array_equal(U.to_np(pr).astype(bool), p2) and int(best[0]) == b2
