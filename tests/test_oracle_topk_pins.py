"""Pins of the top-k state oracle (oracle/topk.py) against brute force and
hand-worked cases."""
import numpy as np

from oracle import topk as OT


def test_select_hand_example_with_ties_and_nan():
    dist = np.array([[0.1, 0.4, 0.4, np.nan, 0.1],
                     [0.2, 0.2, 0.2, 0.2, 0.2]], np.float32)
    idx, val = OT.select(dist, None, 3)
    assert idx.tolist() == [[1, 2, 0], [0, 1, 2]]
    assert np.allclose(val, [[0.4, 0.4, 0.1], [0.2, 0.2, 0.2]])
    idx, val = OT.select(dist, np.array([1, 0]), 2, renormalize=True)
    assert idx.tolist() == [[0, 1], [1, 2]] and np.allclose(val, 0.5)


def test_select_matches_brute_force():
    rng = np.random.default_rng(0)
    dist = np.round(rng.random((200, 12)) * 8) / 8  # many ties
    pixel = rng.integers(0, 200, size=150)
    idx, val = OT.select(dist, pixel, 5)
    for r, p in enumerate(pixel):
        want = sorted(range(12), key=lambda c: (-dist[p, c], c))[:5]
        assert idx[r].tolist() == want
        assert np.array_equal(val[r], dist[p, want].astype(np.float32))
        assert val[r].min() >= np.delete(dist[p], want).max()


def test_update_is_a_convex_step_at_fixed_indices():
    dist = np.array([[0.0, 1.0, 0.5]], np.float32)
    v = OT.update(dist, None, np.array([[2, 1]], np.uint8), np.array([[0.2, 0.4]], np.float32), 0.25)
    assert np.allclose(v, [[0.75 * 0.2 + 0.25 * 0.5, 0.75 * 0.4 + 0.25 * 1.0]])
