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
