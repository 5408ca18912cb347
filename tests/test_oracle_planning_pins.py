"""Pins of the FP64 planning oracle (oracle/planning.py): Fibonacci lattice,
lattice sites, look-at poses and the Eq. 5-7 combination."""
import numpy as np
import pytest
from scipy.special import softmax

from oracle import planning as OP


def test_fibonacci_lattice_closed_form():
    for n in (5, 15, 64):
        d = OP.fibonacci_directions(n)
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
        assert np.allclose(d[:, 2], 1.0 - (2.0 * np.arange(n) + 1.0) / n, atol=0)
        assert abs(d[:, 2].sum()) < 1e-12  # symmetric in z
        az = np.arctan2(d[:, 1], d[:, 0])
        golden = np.pi * (3.0 - np.sqrt(5.0))
        steps = np.mod(np.diff(az) - golden + np.pi, 2 * np.pi) - np.pi
        assert np.allclose(steps, 0.0, atol=1e-12)


def test_sites_hand_example():
    """6 x 5 x 3 voxels of 0.5 m, lattice step 1 m (every second voxel)."""
    nx, ny, nz, vox = 6, 5, 3, 0.5
    before = np.zeros((nz, ny, nx), np.uint8)
    now = np.zeros((nz, ny, nx), np.uint8)
    now[1, 0:3, 0:5] = 1          # newly free on layer 1 ...
    before[1, 0, 0] = 1           # ... except (0, 0), already free before
    now[1, 4, 4] = 1              # on the lattice: (4, 4)
    now[1, 1, 1] = 1              # off the lattice
    now[0, 0, 0] = 1              # another layer
    sites = OP.candidate_sites(now.reshape(-1), before.reshape(-1), (nx, ny, nz), vox, (0.0, 0.0, 0.0), 1.0,
                               0.75, 0.75)
    # layer 1 (centre z = 0.75); lattice ix, iy in {0, 2, 4}; order y then x
    want = [(2, 0), (4, 0), (0, 2), (2, 2), (4, 2), (4, 4)]
    assert sites.shape == (len(want), 3)
    for (ix, iy), p in zip(want, sites):
        assert tuple(p) == ((ix + 0.5) * vox, (iy + 0.5) * vox, 0.75)
    # two heights -> layers 0 and 2 (the lattice in z starts at the first layer in range)
    assert OP.lattice_layers(3, vox, 0.0, 1.0, 0.0, 1.5) == [0, 2]


def test_pose_is_a_look_at_frame():
    p = np.array([1.0, 2.0, 1.5])
    for d in list(OP.fibonacci_directions(15)) + [np.array([1.0, 0.0, 0.0])]:
        v = OP.pose(p, d).astype(np.float64)
        R, t = v[:9].reshape(3, 3), v[9:]
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-6) and np.linalg.det(R) == pytest.approx(1.0, abs=1e-6)
        assert np.allclose(R @ d, [0.0, 0.0, 1.0], atol=1e-6)       # looks along d
        assert np.allclose(R @ p + t, 0.0, atol=1e-5)                # centre at the position
        if abs(d[2]) <= 0.99:
            assert abs(R[0, 2]) < 1e-6                              # right vector horizontal
    R = OP.pose(p, [1.0, 0.0, 0.0])[:9].reshape(3, 3)
    assert np.allclose(R[1], [0.0, 0.0, -1.0], atol=1e-7)           # image down = world down


def test_combine_hand_example():
    n = np.array([10, 30, 0])
    h = np.array([1.0, 2.0, 3.0])
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [1.0, 0.0, 0.0]])
    score, pruned, best = OP.combine(n, h, pos, (0.0, 0.0, 0.0), 1000, prune_fraction=0.02)
    i_geo = np.array([0.25, 0.75, 0.0])
    assert np.allclose(softmax(np.log(n[:2])), i_geo[:2])             # Eq. 5's softmax of log N
    want = (1.0 - softmax([0.0, 5.0, 1.0])) * i_geo * softmax(h)
    assert np.allclose(score, want, rtol=1e-14, atol=0)
    assert list(pruned) == [True, False, True] and best == 1
    # everything pruned
    assert OP.combine([1, 2], [0.0, 0.0], pos[:2], (0, 0, 0), 1000)[2] == -1
