"""Condition estimates of the plain FP64 CG (section 3) against the oracle's
exact spectrum.

The CG's step lengths and residual ratios, recorded on the device, give the
Lanczos tridiagonal whose extreme Ritz values the library reports.  They lie
inside the spectrum of K_hat + gamma I; the largest matches the oracle's
largest eigenvalue closely, the smallest once CG has converged far enough.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _unit_cube(n, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), rng.standard_normal(n)


@pytest.mark.parametrize("sigma,gamma", [(0.1, 1e-2), (0.2, 1e-4), (0.05, 1e-6)])
def test_cg_condition_estimate_matches_spectrum(sigma, gamma):
    from paper_1408_1237_amd import api
    x, y = _unit_cube(1500, 21)
    (w,), (info,) = api.krr_solve([torch.from_numpy(x).cuda()], [sigma], [gamma], [torch.from_numpy(y).cuda()],
                                  mode="cg64", tol=1e-10, max_outer=20000)
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    lo, hi = oracle.eig_extremes(x, sigma, gamma)
    lo_e, hi_e = info["lambda_min_est"], info["lambda_max_est"]
    # Ritz values lie in [lambda_min, lambda_max] up to rounding of order eps ||K||
    slack = 1e-12 * hi
    assert lo - slack <= lo_e <= hi_e <= hi + slack
    assert hi_e == pytest.approx(hi, rel=1e-9)
    assert lo_e == pytest.approx(lo, rel=2e-2)


def test_condition_estimate_only_for_plain_cg():
    from paper_1408_1237_amd import api
    x, y = _unit_cube(600, 22)
    (w,), (info,) = api.krr_solve([torch.from_numpy(x).cuda()], [0.1], [1e-2], [torch.from_numpy(y).cuda()],
                                  mode="fgmres")
    assert info["status"] == 0
    assert info["lambda_min_est"] == 0.0 and info["lambda_max_est"] == 0.0


def test_condition_estimate_of_a_truncated_run_is_a_lower_bound():
    # CG stopped early: lambda_max already accurate, lambda_min from above
    from paper_1408_1237_amd import api
    x, y = _unit_cube(1500, 23)
    (w,), (info,) = api.krr_solve([torch.from_numpy(x).cuda()], [0.2], [1e-6], [torch.from_numpy(y).cuda()],
                                  mode="cg64", tol=1e-10, max_outer=40)
    assert info["status"] == 1 and info["outer_iters"] == 40
    lo, hi = oracle.eig_extremes(x, 0.2, 1e-6)
    assert info["lambda_max_est"] == pytest.approx(hi, rel=1e-6)
    assert info["lambda_min_est"] >= lo - 1e-12 * hi
    assert info["lambda_max_est"] / info["lambda_min_est"] <= hi / lo
