"""GPR prediction (section 2.1) on the GPU: posterior mean (eq. GPR_mean) and
variance against the oracle's Cholesky-based prediction (pinned to
scikit-learn's GaussianProcessRegressor)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kernel", ["gauss", "matern32"])
def test_predict_matches_oracle(kernel):
    from paper_1408_1237_amd import api
    x = workloads.random_points(160, 1500, 3, 1.0)
    xs = np.concatenate([workloads.random_points(161, 36, 3, 1.0), np.full((1, 3), 50.0)])  # 37: ragged batches
    y = np.sin(3 * x[:, 0]) + 0.1 * workloads.random_vector(162, 1500)
    sigma, gamma = 0.3, 1e-2
    if kernel == "gauss":
        w = oracle.direct_solve(x, sigma, gamma, y)
    else:
        w = oracle.matern_direct_solve(x, sigma, gamma, y)
    mean, var, infos = api.krr_predict(_t(x), _t(xs), sigma, gamma, _t(w), kernel=kernel, tol=1e-10,
                                       max_outer=5000, restart_m=50, inner_maxit=20)
    m_ref, v_ref = oracle.predict(x, xs, sigma, gamma, y, kernel=kernel)
    mean, var = mean.cpu().numpy(), var.cpu().numpy()
    assert np.allclose(mean, m_ref, rtol=1e-9, atol=1e-10)
    assert len(infos) == 37 and all(i["status"] == 0 for i in infos)
    assert np.max(np.abs(var - v_ref)) <= 1e-6
    assert var[-1] == pytest.approx(1.0, abs=1e-12) and abs(mean[-1]) <= 1e-12  # far from every training point


def test_predict_mean_only_at_kriging_scale():
    from paper_1408_1237_amd import api
    p = workloads.kriging(n=20000)
    xs = workloads.random_points(163, 2000, 3, 10.0)
    w = workloads.random_vector(164, p.n)
    mean, var, _ = api.krr_predict(_t(p.x), _t(xs), p.sigma, p.gamma, _t(w), want_var=False)
    assert var is None
    want = oracle.mvp(xs, p.sigma, w, xs=p.x)
    assert np.linalg.norm(mean.cpu().numpy() - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("kernel", ["gauss", "matern32"])
def test_predict_mean_large_d(kernel):
    # the posterior mean at d = 20 (cross products through the large-d VALU
    # kernels in FP64) against the oracle's Cholesky prediction
    from paper_1408_1237_amd import api
    d = 20
    x = workloads.random_points(170, 800, d, 1.0, kind="normal")
    xs = workloads.random_points(171, 45, d, 1.0, kind="normal")
    y = np.tanh(x[:, 0] - x[:, 1]) + 0.1 * workloads.random_vector(172, 800)
    sigma, gamma = 0.6 * np.sqrt(d), 1e-2
    if kernel == "gauss":
        w = oracle.direct_solve(x, sigma, gamma, y)
    else:
        w = oracle.matern_direct_solve(x, sigma, gamma, y)
    mean, var, _ = api.krr_predict(_t(x), _t(xs), sigma, gamma, _t(w), want_var=False, kernel=kernel)
    m_ref, _ = oracle.predict(x, xs, sigma, gamma, y, kernel=kernel)
    assert var is None
    assert np.allclose(mean.cpu().numpy(), m_ref, rtol=1e-9, atol=1e-10)
