"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/sgr.h declares, and rejects invalid arguments on
the host before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2506_00225_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2506_00225_amd import build
        build.build()
    _lib.lib()
    return _lib


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(sgr_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 10
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(L.EXPORTS) == set(names)


def _cam(w=64, h=48, f=50.0):
    from paper_2506_00225_amd import _lib
    return _lib.sgr_camera((ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1), (ctypes.c_float * 3)(0, 0, 0), f, f,
                           w / 2, h / 2, w, h)


def _cfg(C=16, k=3, **kw):
    from paper_2506_00225_amd import make_config
    return make_config(C, k, **kw)


def _cams(*cs):
    from paper_2506_00225_amd import _lib
    arr = (_lib.sgr_camera * len(cs))()
    for i, c in enumerate(cs):
        arr[i] = c
    return arr


def test_workspace_size_valid_and_layout(L):
    cams = _cams(_cam(), _cam(160, 120, 80.0))
    size = L.sgr_workspace_size(1000, cams, 2, _cfg(), 50000)
    assert size > 0 and size % 256 == 0
    lay = L.sgr_workspace_layout(1000, cams, 2, _cfg(), 50000)
    assert lay.total_bytes == size
    assert lay.counters == 0
    assert lay.num_tiles == 4 * 3 + 10 * 8
    assert lay.num_pixels == 64 * 48 + 160 * 120
    assert lay.vn == 2000
    offs = [lay.views, lay.proj_count, lay.proj_zbits, lay.pair_rec, lay.pair_lin, lay.order, lay.sorted_keys,
            lay.sorted_vals, lay.key_owner, lay.ranges, lay.tile_offsets]
    assert all(o % 256 == 0 and 0 < o < size for o in offs)


@pytest.mark.parametrize("bad", [
    dict(n=-1), dict(V=0), dict(cap=0), dict(C=0), dict(C=257), dict(k=0), dict(k=33),
    dict(alpha_min=0.0), dict(alpha_max=1.0), dict(t_min=0.0), dict(z_near=0.0), dict(lowpass=-1.0),
    dict(width=0), dict(fx=float("nan")), dict(n=1 << 30, V=4),
])
def test_invalid_arguments_rejected(L, bad):
    n, V, cap = bad.get("n", 10), bad.get("V", 1), bad.get("cap", 100)
    cfgkw = {k: v for k, v in bad.items() if k in ("alpha_min", "alpha_max", "t_min", "z_near", "lowpass")}
    cfg = _cfg(C=bad.get("C", 16), k=bad.get("k", 3), **cfgkw)
    cam = _cam(w=bad.get("width", 64), f=bad.get("fx", 50.0))
    cams = _cams(*([cam] * max(V, 1)))
    assert L.sgr_workspace_size(n, cams, V, cfg, cap) == 0


def test_unsupported_tile(L):
    cfg = _cfg()
    cfg.tile_w = 8
    with pytest.raises(L.SgrError) as e:
        L.sgr_workspace_layout(10, _cams(_cam()), 1, cfg, 100)
    assert e.value.status == L.SGR_EUNSUPPORTED


def test_accumulator_placement_validated(L):
    cfg = _cfg(C=130, k=3)
    cfg.sem_accumulators = L.SGR_ACC_REGISTERS  # 130 classes exceed the register accumulators
    with pytest.raises(L.SgrError) as e:
        L.sgr_workspace_layout(10, _cams(_cam()), 1, cfg, 100)
    assert e.value.status == L.SGR_EUNSUPPORTED
    cfg.sem_accumulators = 3
    assert L.sgr_workspace_size(10, _cams(_cam()), 1, cfg, 100) == 0
    for acc in (L.SGR_ACC_AUTO, L.SGR_ACC_LDS):
        cfg.sem_accumulators = acc
        assert L.sgr_workspace_size(10, _cams(_cam()), 1, cfg, 100) > 0
    for passes, ok in ((-1, False), (0, True), (1, True), (4, True), (5, False)):
        cfg.sem_passes = passes
        assert (L.sgr_workspace_size(10, _cams(_cam()), 1, cfg, 100) > 0) == ok, passes


def test_calls_validate_before_any_device_work(L):
    """Bad workspace or pointers come back as SGR_EINVAL from the host layer
    (these calls never reach HIP, so they run without a GPU)."""
    cams = _cams(_cam())
    cfg = _cfg()
    g = L.sgr_gaussians(10, None, None, None, None, None, None, None)
    assert L.sgr_project(g, cams, 1, cfg, 100, None, 0, None) == L.SGR_EINVAL
    size = L.sgr_workspace_size(10, cams, 1, cfg, 100)
    buf = (ctypes.c_uint8 * (size + 512))()
    addr = (ctypes.addressof(buf) + 255) // 256 * 256
    # null Gaussian arrays with n > 0
    assert L.sgr_project(g, cams, 1, cfg, 100, addr, size, None) == L.SGR_EINVAL
    arr = np.zeros(40, np.float32)
    p = arr.ctypes.data
    g = L.sgr_gaussians(10, p, p, p, p, p, p, p)
    # workspace too small / misaligned
    assert L.sgr_project(g, cams, 1, cfg, 100, addr, size - 1, None) == L.SGR_EINVAL
    assert L.sgr_project(g, cams, 1, cfg, 100, addr + 4, size, None) == L.SGR_EINVAL
    assert L.sgr_render_forward(g, cams, 1, cfg, 100, None, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_score_views(g, cams, 1, cfg, 100, None, None, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_score_maps(None, None, 4, 4, 16, None, None, None, 0, None) == L.SGR_EINVAL
    assert L.sgr_score_maps_workspace_size(0, 4) == 0
    assert L.sgr_score_maps_noalloc(None, None, 4, 4, 16, None, None, None) == L.SGR_EINVAL
    # fused gather + Adam: no segments, a bad step, a segment of the wrong size
    segs = (L.sgr_adam_segment * 6)()
    gw = L.sgr_gaussians(10, *([ctypes.c_void_p(256)] * 7))
    lib = L.lib()
    assert lib.sgr_render_backward_gather_adam(gw, cams, 1, cfg, 100, None, 1e-3, 0.9, 0.999, 1e-8, 1,
                                               addr, size, None) == L.SGR_EINVAL
    assert lib.sgr_render_backward_gather_adam(gw, cams, 1, cfg, 100, segs, 1e-3, 0.9, 0.999, 1e-8, 0,
                                               addr, size, None) == L.SGR_EINVAL
    one = ctypes.c_void_p(256)
    for i, n in enumerate((30, 30, 40, 10, 30, 30)):
        segs[i] = L.sgr_adam_segment(one, None, one, one, n, 0.0, 1.0)
    segs[5].n = 29  # k n = 30 expected
    assert lib.sgr_render_backward_gather_adam(gw, cams, 1, cfg, 100, segs, 1e-3, 0.9, 0.999, 1e-8, 1,
                                               addr, size, None) == L.SGR_EINVAL
    one = ctypes.c_void_p(256)  # never dereferenced: each call below returns before any device work
    assert L.sgr_score_maps_noalloc(one, one, 0, 4, 16, one, one, None) == L.SGR_EINVAL
    assert L.sgr_score_maps_noalloc(one, one, 4, 4, 0, one, one, None) == L.SGR_EINVAL
    assert L.sgr_score_maps_noalloc(one, one, 4097, 4096, 16, one, one, None) == L.SGR_EUNSUPPORTED
    # fused forward + loss: missing views, config or loss output; negative weights
    lv = (L.sgr_loss_view * 1)()
    lc = L.sgr_loss_config(1.0, 0.5, 1.0, 1.0, 0.99, 1e-6, 0.8, 0.2, 0.0, 1e-8)
    out = np.zeros(1, np.float64).ctypes.data
    assert L.sgr_render_forward_loss(g, cams, 1, cfg, 100, None, None, lc, out, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_render_forward_loss(g, cams, 1, cfg, 100, None, lv, lc, None, addr, size, None) == L.SGR_EINVAL
    bad = L.sgr_loss_config(1.0, -0.5, 1.0, 1.0, 0.99, 1e-6, 0.8, 0.2, 0.0, 1e-8)
    assert L.sgr_render_forward_loss(g, cams, 1, cfg, 100, None, lv, bad, out, addr, size, None) == L.SGR_EINVAL
    bad = L.sgr_loss_config(1.0, 0.5, 1.0, 1.0, 0.99, 0.0, 0.8, 0.2, 0.0, 1e-8)
    assert L.sgr_render_forward_loss(g, cams, 1, cfg, 100, None, lv, bad, out, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_render_forward_loss(g, cams, 1, cfg, 100, None, lv, lc, out, addr, size - 1, None) == L.SGR_EINVAL


def test_status_strings(L):
    for s in range(5):
        assert isinstance(L.sgr_status_string(s), str) and L.sgr_status_string(s)
    assert L.sgr_status_string(99) == "unknown status"


def test_capacity_needed_exceeds_small_capacity_per_oracle():
    """The key count the oracle finds for config 0 is what a capacity check
    must compare against: a capacity below it is an overflow (the GPU test
    checks that the device reports it)."""
    from oracle import oracle as O
    from paper_2506_00225_amd import scenes
    sc = scenes.tiny_scene()
    pr = O.project(sc.means, sc.scales, sc.quats, sc.opacity, sc.cameras[0], O.config_array())
    keys, _, _ = O.reference_keys([pr], sc.cameras)
    assert len(keys) > 1000


def test_planning_calls_validate_on_the_host(L):
    grid = L.sgr_grid(40, 32, 12, 0.25, (ctypes.c_float * 3)(0.0, 0.0, 0.0))
    samp = L.sgr_sampling(1.0, 5, 1.5, 1.5)
    size = L.sgr_candidates_workspace_size(grid, samp)
    assert size > 0 and size % 256 == 0
    for bad_grid, bad_samp in ((L.sgr_grid(0, 32, 12, 0.25, (ctypes.c_float * 3)()), samp),
                               (L.sgr_grid(40, 32, 12, 0.0, (ctypes.c_float * 3)()), samp),
                               (grid, L.sgr_sampling(0.0, 5, 1.5, 1.5)),
                               (grid, L.sgr_sampling(1.0, 0, 1.5, 1.5)),
                               (grid, L.sgr_sampling(1.0, 5, 2.0, 1.0))):
        assert L.sgr_candidates_workspace_size(bad_grid, bad_samp) == 0
    buf = (ctypes.c_uint8 * (size + 512))()
    addr = (ctypes.addressof(buf) + 255) // 256 * 256
    cnt = np.zeros(1, np.int64).ctypes.data
    # missing grid bytes / count, workspace too small
    assert L.sgr_generate_candidates(grid, None, None, samp, 0, None, None, cnt, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_generate_candidates(grid, addr, None, samp, 0, None, None, None, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_generate_candidates(grid, addr, None, samp, 0, None, None, cnt, addr, size - 1, None) == L.SGR_EINVAL
    assert L.sgr_generate_candidates(grid, addr, None, samp, 4, None, None, cnt, addr, size, None) == L.SGR_EINVAL
    p = np.zeros(16, np.float64).ctypes.data
    assert L.sgr_combine_scores(0, p, p, p, (0, 0, 0), 100, 0.005, p, p, p, None) == L.SGR_EINVAL
    assert L.sgr_combine_scores(2, p, p, p, (0, 0, 0), 0, 0.005, p, p, p, None) == L.SGR_EINVAL
    assert L.sgr_combine_scores(2, p, p, p, (0, 0, float("nan")), 100, 0.005, p, p, p, None) == L.SGR_EINVAL
    assert L.sgr_combine_scores(2, None, p, p, (0, 0, 0), 100, 0.005, p, p, p, None) == L.SGR_EINVAL
    g = L.sgr_gaussians(10, p, p, p, p, p, p, p)
    assert L.sgr_score_poses(g, None, 2, p, _cfg(), 100, p, p, addr, size, None) == L.SGR_EINVAL
    assert L.sgr_score_poses(g, _cams(_cam()), 2, None, _cfg(), 100, p, p, addr, size, None) == L.SGR_EINVAL
