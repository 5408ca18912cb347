"""Host-side checks of the benchmark's roofline bookkeeping (no GPU)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _out(**stage):
    base = {"proj": 0.2, "bin": 0.15, "fwd": 0.27, "bwd_tiles": 0.48, "bwd_gather": 0.15, "adam": 0.14}
    base.update(stage)
    return {"pixels": 1200 * 680, "C": 102, "k": 16, "keys": 2_500_000, "nvis": 280_000, "n": 1_000_000,
            "blends": 5.0e7, "stage_ms": base}


def test_compositing_stage_is_reported_against_the_alu_peak():
    dom, r = bench.roofline(_out())
    assert dom == "bwd_tiles" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["flops_per_blend"] == 12 + 45  # an FMA counted as 2 flops
    assert abs(r["achieved"] - 5.0e7 * r["flops_per_blend"] / 0.48e-3 / 1e12) < 1e-3
    assert abs(r["frac"] - r["achieved"] / bench.FP32_PEAK_TFLOPS) < 1e-4
    assert abs(r["frac_unpacked"] - r["achieved"] / bench.FP32_UNPACKED_TFLOPS) < 1e-4
    assert 0 < r["hbm_frac"] < 1


def test_forward_dominant_uses_forward_count():
    dom, r = bench.roofline(_out(fwd=0.9))
    assert dom == "fwd" and r["flops_per_blend"] == 12 + 14 and r["kernel"] == "render_fwd_label_kernel"


def test_memory_stage_is_reported_against_hbm():
    dom, r = bench.roofline(_out(bwd_gather=2.0))
    assert dom == "bwd_gather" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["frac"] - r["achieved"] / bench.HBM_PEAK_GBS) < 1e-4


def test_path_hbm_fraction_uses_both_byte_counts():
    out = _out()
    out["fwd_bwd_ms"] = 1.0
    h = bench.hbm_path(out)
    P, C, k, K, Nv, n = 1200 * 680, 102, 16, 2_500_000, 280_000, 1_000_000
    want = (44 + 36 + 8) * n + 40 * K + (48 + 5 * k) * Nv + P * (5 + C) * 4 + 8 * P \
        + P * (5 + C) * 4 + 8 * P + 4 * K + (48 + 5 * k) * Nv + (40 + 4 * k + 72 + 44) * n
    assert h["scope_formula_bytes"] == want
    assert abs(h["scope_formula_frac"] - want / 1e-3 / 8e12) < 1e-4
    assert h["fused_path_bytes"] < h["scope_formula_bytes"]  # the class maps stay on chip
    assert abs(h["target_ms_at_half_peak"] - want / 4e12 * 1e3) < 1e-4
