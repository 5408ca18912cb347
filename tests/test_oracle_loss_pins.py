"""Pins of the FP64 mapping-loss oracle (oracle/loss.py) against closed
forms, textbook identities, library routines and finite differences."""
import numpy as np
import pytest
from scipy.spatial.distance import cosine as scipy_cosine_distance
from scipy.stats import entropy as scipy_entropy

from oracle import loss as OL


def test_entropy_matches_scipy_and_handles_zeros():
    rng = np.random.default_rng(0)
    g = rng.dirichlet(np.ones(7), size=5)
    g[0, 3] = 0.0
    g[0] /= g[0].sum()
    for row, h in zip(g, OL.entropy(g)):
        assert h == pytest.approx(scipy_entropy(row), rel=1e-12)


def test_hellinger_identity_and_extremes():
    """D_HD^2 = 1 - sum sqrt(g q) for distributions (e = 0); identical
    distributions give 0, disjoint one-hots give 1."""
    rng = np.random.default_rng(1)
    g, q = rng.dirichlet(np.ones(9), size=4), rng.dirichlet(np.ones(9), size=4)
    d = OL.hellinger(g, q, 0.0)
    assert np.allclose(d ** 2, 1.0 - np.sqrt(g * q).sum(-1), rtol=0, atol=1e-14)
    assert np.allclose(OL.hellinger(g, g, 1e-8), 0.0, atol=0)
    e0, e1 = np.eye(5)[0], np.eye(5)[1]
    assert OL.hellinger(e0, e1, 0.0) == pytest.approx(1.0, abs=1e-15)


def test_semantic_term_closed_forms_and_scipy_cosine():
    k = 4
    # q = g: no loss
    g = np.array([0.7, 0.2, 0.1, 0.0, 0.0])
    v, gr, mask, _ = OL.semantic_term(g, g.copy(), k)
    assert mask and v == pytest.approx(0.0, abs=1e-12)
    # disjoint one-hots: 0.8 D_HD + 0.2 (1 - 0), D_HD -> 1 as e -> 0
    v, _, mask, _ = OL.semantic_term(np.eye(5)[0], np.eye(5)[1], k, sqrt_eps=0.0)
    assert mask and v == pytest.approx(1.0, abs=1e-12)
    # cosine part against scipy's cosine distance
    rng = np.random.default_rng(2)
    g = rng.dirichlet(np.ones(6) * 0.2)
    q = rng.random(6)
    v, _, mask, H = OL.semantic_term(g, q, 6, lambda_hd=0.0, lambda_cos=1.0)
    assert H < np.log(6) and mask
    assert v == pytest.approx(scipy_cosine_distance(g, q), rel=1e-12)


def test_entropy_mask_threshold_is_ln_k_strict():
    k = 4
    uni_k = np.full(8, 0.0)
    uni_k[:k] = 1.0 / k           # H = ln k: not below tau, unsupervised
    uni_km1 = np.full(8, 0.0)
    uni_km1[:k - 1] = 1.0 / (k - 1)
    q = np.full(8, 0.1)
    assert not OL.semantic_term(uni_k, q, k)[2]
    assert OL.semantic_term(uni_km1, q, k)[2]
    # an empty rendered distribution has no cosine: no semantic term
    assert not OL.semantic_term(uni_km1, np.zeros(8), k)[2]


def _maps(rng, H, W, C):
    return {"rgb": rng.random((H, W, 3)), "depth": rng.random((H, W)) * 4 + 0.5,
            "sil": np.where(rng.random((H, W)) < 0.5, 0.995, 0.9) + rng.random((H, W)) * 1e-3,
            "sem": rng.random((H, W, C)) * 0.2 + 0.01}


@pytest.mark.parametrize("sem", ["ce", "hd_cos", "none"])
def test_mapping_loss_gradient_matches_central_differences(sem):
    rng = np.random.default_rng(3)
    H, W, C, k = 3, 4, 6, 3
    maps = _maps(rng, H, W, C)
    tg = {"rgb": rng.random((H, W, 3)), "depth": rng.random((H, W)) * 4 + 0.5}
    if sem == "ce":
        tg["label"] = rng.integers(0, C, size=(H, W))
    elif sem == "hd_cos":
        tg["sem"] = rng.dirichlet(np.ones(C) * 0.1, size=(H, W))   # peaked: most pixels under ln k
    loss, grads, flags = OL.mapping_loss(maps, tg, C, k)
    assert not flags.any()
    h = 1e-6
    for key in ("rgb", "depth", "sil", "sem"):
        it = np.nditer(maps[key], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            mp, mm = {a: b.copy() for a, b in maps.items()}, {a: b.copy() for a, b in maps.items()}
            mp[key][idx] += h
            mm[key][idx] -= h
            fd = (OL.mapping_loss(mp, tg, C, k)[0] - OL.mapping_loss(mm, tg, C, k)[0]) / (2 * h)
            assert grads[key][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (key, idx)


def test_mapping_loss_hand_example():
    """One pixel: S = 0.995 > 0.99, so depth and colour count."""
    maps = {"rgb": np.array([[[0.5, 0.5, 0.5]]]), "depth": np.array([[2.0]]), "sil": np.array([[0.995]]),
            "sem": np.array([[[0.25, 0.5, 0.0]]])}
    tg = {"rgb": np.array([[[0.0, 1.0, 0.5]]]), "depth": np.array([[3.0]]), "label": np.array([[1]])}
    loss, g, _ = OL.mapping_loss(maps, tg, 3, 2)
    # 1.0*|2-3| + 0.5*(0.5 + 0.5 + 0) + 1.0*|0.995-1| - ln 0.5
    assert loss == pytest.approx(1.0 + 0.5 + 0.005 + np.log(2.0), rel=1e-12)
    assert g["depth"][0, 0] == -1.0 and list(g["rgb"][0, 0]) == [0.5, -0.5, 0.0]
    assert g["sil"][0, 0] == -1.0 and list(g["sem"][0, 0]) == [0.0, -2.0, 0.0]
