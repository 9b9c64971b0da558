"""Gradient pass and the differentiable solve on the GPU.

kmvp_grad is compared with the oracle's explicit gradient (same lambda and w);
the exact invariants sum_i dl/dx_i = 0 and sum_i x_i . dl/dx_i + dl/dlog sigma = 0
are checked at the full GP-regression shape; the autograd gradient of
l = y^T K^{-1} y is compared with FP64 central finite differences of direct
(Cholesky) solves.  Bars: FP64 pass 1e-11 relative, FP32 pass 1e-5 relative
(random lambda and w, so the row sums do not cancel beyond a few digits).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


BAR = {"fp64": 1e-11, "fp32": 1e-5}


def _grad(x, sigma, gamma, lam, w, same=False, prec="fp64"):
    from paper_1408_1237_amd import api
    lt = _t(lam)
    wt = lt if same else _t(w)
    gx, gs, gg = api.kmvp_grad(_t(x), sigma, gamma, lt, wt, prec=prec)
    torch.cuda.synchronize()
    return gx.cpu().numpy(), float(gs), float(gg)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,d", [(1, 2), (3, 1), (300, 2), (700, 3), (1000, 8), (513, 16), (400, 33)])
def test_grad_matches_oracle(n, d, prec):
    x = workloads.random_points(40 + n, n, d, 1.0, kind="normal")
    lam = workloads.random_vector(41 + n, n)
    w = workloads.random_vector(42 + n, n)
    sigma, gamma = 0.8 * np.sqrt(d), 0.03
    gx, gs, gg = _grad(x, sigma, gamma, lam, w, prec=prec)
    ox, os_, og = oracle.grad(x, sigma, gamma, lam, w)
    scale = max(np.linalg.norm(ox), 1e-300)
    assert np.linalg.norm(gx - ox) / scale <= BAR[prec]
    assert gs == pytest.approx(os_, rel=BAR[prec], abs=0.1 * BAR[prec] * scale)
    assert gg == pytest.approx(og, rel=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_grad_same_lambda_and_w(prec):
    x = workloads.random_points(50, 800, 4, 1.0, kind="normal")
    w = workloads.random_vector(51, 800)
    gx, gs, gg = _grad(x, 1.5, 0.01, w, w, same=True, prec=prec)
    ox, os_, og = oracle.grad(x, 1.5, 0.01, w, w)
    assert np.linalg.norm(gx - ox) / np.linalg.norm(ox) <= BAR[prec]
    # d/dlog sigma is a sum of N^2 terms lam_i w_j K_ij |x_i - x_j|^2 of both
    # signs (random w: the sum is about 1/80 of the sum of their magnitudes); an
    # FP32 accumulation is held to the bar relative to that magnitude sum, which
    # the oracle gives for |w| (every term positive), FP64 to the sum itself
    scale = abs(oracle.grad(x, 1.5, 0.01, np.abs(w), np.abs(w))[1]) if prec == "fp32" else abs(os_)
    assert abs(gs - os_) <= BAR[prec] * scale


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_grad_invariants_full_gp_shape(prec):
    # N = 2e5, d = 16; exact identities for any lambda, w
    p = workloads.gp_regression()
    lam = workloads.random_vector(52, p.n)
    w = workloads.random_vector(53, p.n)
    gx, gs, gg = _grad(p.x, p.sigma, p.gamma, lam, w, prec=prec)
    tot = np.abs(gx).sum(axis=0)
    assert np.all(np.abs(gx.sum(axis=0)) <= BAR[prec] * tot)
    xs = (p.x * gx).sum()
    assert abs(xs + gs) <= BAR[prec] * (np.abs(p.x * gx).sum() + abs(gs))
    assert gg == pytest.approx(-p.gamma * lam @ w, rel=1e-12)


def test_grad_bad_precision_rejected():
    from paper_1408_1237_amd import api, native
    x = _t(workloads.random_points(60, 100, 2, 1.0))
    v = _t(workloads.random_vector(61, 100))
    with pytest.raises(native.KrrError):
        api.kmvp_grad(x, 1.0, 0.1, v, v, prec="bf16")


def test_autograd_matches_finite_differences():
    from paper_1408_1237_amd import autograd
    p = workloads.gp_regression(n=400, d=4)
    sigma, gamma = 2.0, 0.05
    x = _t(p.x).requires_grad_(True)
    y = _t(p.y).requires_grad_(True)
    ls = torch.tensor(np.log(sigma), dtype=torch.float64, device="cuda", requires_grad=True)
    lg = torch.tensor(np.log(gamma), dtype=torch.float64, device="cuda", requires_grad=True)
    w = autograd.krr_solve(x, y, ls, lg, tol=1e-12, inner_prec="fp64", inner_maxit=50, restart_m=200)
    loss = (y * w).sum()
    gx, gy, gls, glg = torch.autograd.grad(loss, (x, y, ls, lg))

    def l(xx, s, g):
        return float(p.y @ oracle.direct_solve(xx, s, g, p.y))

    h = 1e-6
    fd_s = (l(p.x, sigma * np.exp(h), gamma) - l(p.x, sigma * np.exp(-h), gamma)) / (2 * h)
    fd_g = (l(p.x, sigma, gamma * np.exp(h)) - l(p.x, sigma, gamma * np.exp(-h))) / (2 * h)
    assert float(gls) == pytest.approx(fd_s, rel=1e-5)
    assert float(glg) == pytest.approx(fd_g, rel=1e-5)
    gxn = gx.cpu().numpy()
    for i, t in [(0, 0), (17, 3), (399, 1)]:
        xp, xm = p.x.copy(), p.x.copy()
        xp[i, t] += h
        xm[i, t] -= h
        fd = (l(xp, sigma, gamma) - l(xm, sigma, gamma)) / (2 * h)
        assert gxn[i, t] == pytest.approx(fd, rel=1e-4, abs=1e-6 * np.abs(gxn).max())
    # dl/dy = 2 w for l = y^T K^{-1} y
    assert np.allclose(gy.cpu().numpy(), 2 * w.detach().cpu().numpy(), rtol=1e-9, atol=1e-12)
