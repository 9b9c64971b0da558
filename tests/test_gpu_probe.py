"""The issue-rate probe behind the product rooflines (GPU)."""
import pytest

pytestmark = pytest.mark.gpu

SIMD_CYCLES_S = 256 * 4 * 2.4e9


def test_probe_rates_within_unit_count_bounds():
    from paper_1408_1237_amd import api
    r = api.probe_issue_rates()
    assert all(v > 0 for v in r.values())
    # nothing can beat the issue limits derived from the unit counts
    assert r["fma_lane_ops_s"] <= 1.05 * SIMD_CYCLES_S * 16
    assert r["mfma_pairs_s"] <= 1.05 * SIMD_CYCLES_S * 256 / 32
    assert r["exp_fma_pairs_s"] <= 1.05 * SIMD_CYCLES_S * 16
    assert r["mg_mix_pairs_s"] <= 1.05 * min(r["exp_fma_pairs_s"], r["mfma_pairs_s"])
    # the split-f16 mix: one 32x32x16 f16 operation per 1024 pairs, which also
    # need 16 exp2 (8 cycles) and 16 FMAs (4 cycles) per lane on the VALU
    assert r["mh_mix_pairs_s"] <= 1.05 * SIMD_CYCLES_S * 1024 / (16 * (8 + 4))
    assert r["mh_mix_pairs_s"] > r["mg_mix_pairs_s"]
    # FP64 exp2 takes at least 13 FP64 VALU instructions (4 cycles each) per pair
    assert r["exp64_fma_pairs_s"] <= 1.05 * SIMD_CYCLES_S * 64 / (13 * 4)
