"""The scoring entry point that allocates nothing (sgr_score_maps_noalloc)
against sgr_score_maps with a caller workspace, through the C ABI: two calls
in a row on the library's static scratch, the second with a smaller view
(so stale partial sums of the first call would show), each equal bit for
bit to the workspace path on the same maps."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2506_00225_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def _maps(seed, W, H, C):
    """Dense class sums and contributor counts of one view: rows of random
    mass in [0, 1] over C classes, with about a fifth of the pixels empty."""
    rng = np.random.default_rng(seed)
    sem = rng.random((H, W, C)).astype(np.float32)
    sem *= (rng.random((H, W, 1)) / sem.sum(-1, keepdims=True)).astype(np.float32)
    nc = rng.integers(1, 40, size=(H, W)).astype(np.int32)
    empty = rng.random((H, W)) < 0.2
    nc[empty] = 0
    sem[empty] = 0
    return torch.from_numpy(sem).cuda().contiguous(), torch.from_numpy(nc).cuda().contiguous()


def _with_workspace(sem, nc, C):
    H, W = nc.shape
    need = L.sgr_score_maps_workspace_size(W, H)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    ne = torch.empty(1, dtype=torch.int32, device="cuda")
    es = torch.empty(1, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sgr_score_maps(ctypes.c_void_p(sem.data_ptr()), ctypes.c_void_p(nc.data_ptr()), W, H, C,
                            ctypes.c_void_p(ne.data_ptr()), ctypes.c_void_p(es.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), need, st) == L.SGR_OK
    return ne, es


def _no_alloc(sem, nc, C):
    H, W = nc.shape
    ne = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    es = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sgr_score_maps_noalloc(ctypes.c_void_p(sem.data_ptr()), ctypes.c_void_p(nc.data_ptr()), W, H, C,
                                    ctypes.c_void_p(ne.data_ptr()), ctypes.c_void_p(es.data_ptr()), st) == L.SGR_OK
    return ne, es


def test_no_alloc_scoring_equals_workspace_scoring_twice():
    print("[case] score_maps_noalloc: 640x480 C=102, then 160x120 C=40", flush=True)
    for seed, W, H, C in ((0, 640, 480, 102), (1, 160, 120, 40)):
        sem, nc = _maps(seed, W, H, C)
        ne_a, es_a = _no_alloc(sem, nc, C)
        ne_b, es_b = _with_workspace(sem, nc, C)
        torch.cuda.synchronize()
        assert int(ne_a[0]) == int(ne_b[0]) == int((nc == 0).sum())
        assert es_a.cpu().numpy().tobytes() == es_b.cpu().numpy().tobytes(), (float(es_a[0]), float(es_b[0]))
        assert np.isfinite(float(es_a[0])) and float(es_a[0]) > 0


def test_no_alloc_rejects_a_view_beyond_its_scratch():
    sem, nc = _maps(2, 16, 16, 8)
    ne = torch.empty(1, dtype=torch.int32, device="cuda")
    es = torch.empty(1, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # checked on the host before anything is enqueued; the pointers are never read
    W, H = 4097, 4096
    assert W * H > L.SGR_NOALLOC_MAX_PIXELS
    assert L.sgr_score_maps_noalloc(ctypes.c_void_p(sem.data_ptr()), ctypes.c_void_p(nc.data_ptr()), W, H, 8,
                                    ctypes.c_void_p(ne.data_ptr()), ctypes.c_void_p(es.data_ptr()),
                                    st) == L.SGR_EUNSUPPORTED
    torch.cuda.synchronize()
