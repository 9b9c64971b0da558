"""Flexible CG (sections 4.2 and 5.4) on the GPU against the oracle.

The GPU keeps restart_m direction slots (each new direction is K-orthogonalised
against up to restart_m - 1 previous ones), the oracle's window is mmax =
restart_m - 1.  Iteration counts are compared loosely (rounding decides them in
ill-conditioned cases); solutions against the Cholesky solve within kappa * tol.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _solve(p, mode="fcg", **opts):
    from paper_1408_1237_amd import api
    (w,), (info,) = api.krr_solve([_t(p.x)], [p.sigma], [p.gamma], [_t(p.y)], mode=mode, **opts)
    return w.cpu().numpy(), info


@pytest.mark.parametrize("inner_prec", ["fp64", "fp32", "bf16"])
def test_fcg_plain_small_paper_settings(inner_prec):
    # the paper's FCG settings on the unit-square set: delta = 1e-4, inner tolerance 1e-4
    p = workloads.plain_small()
    w, info = _solve(p, inner_prec=inner_prec, delta=1e-4, inner_tol=1e-4, inner_maxit=200, restart_m=31,
                     max_outer=500)
    assert info["status"] == 0 and info["relres_true"] <= 1e-6
    assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w) <= 1.01e-6
    ref = oracle.fcg(p.x, p.sigma, p.gamma, p.y, mmax=30, max_outer=500, delta=1e-4, inner_tol=1e-4,
                     inner_maxit=200)
    assert ref["status"] == 0
    lo, hi = 0.6 * ref["outer"], 1.6 * ref["outer"] + 2
    assert lo <= info["outer_iters"] <= hi


def test_fcg_without_preconditioner_matches_cg_and_cholesky():
    p = workloads.plain_small(n=600)
    w, info = _solve(p, inner="none", restart_m=8, max_outer=5000)
    assert info["status"] == 0
    ws = oracle.direct_solve(p.x, p.sigma, p.gamma, p.y)
    K = oracle.kernel_matrix(p.x, p.sigma) + p.gamma * np.eye(p.n)
    assert np.linalg.norm(w - ws) <= np.linalg.cond(K) * 1e-6 * np.linalg.norm(ws)
    c = oracle.cg(p.x, p.sigma, p.gamma, p.y, 5000, 1e-6)
    assert abs(info["outer_iters"] - c[2]) <= 0.25 * c[2] + 3


def test_fcg_not_converged_and_matern():
    w, info = _solve(workloads.plain_small(), inner_maxit=3, max_outer=4)
    assert info["status"] == 1 and info["outer_iters"] == 4 and 1e-6 < info["relres_true"] < 1.0
    pm = workloads.matern_classification(n=1200, d=3)
    w, info = _solve(pm, kernel="matern32", inner_maxit=30, restart_m=20, max_outer=500)
    assert info["status"] == 0
    r = pm.y - oracle.matern_mvp(pm.x, pm.sigma, w, shift=pm.gamma)
    assert np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(pm.y)


def test_fcg_several_systems():
    from paper_1408_1237_amd import api
    probs = [workloads.plain_small(seed=140 + k, n=500 + 200 * k) for k in range(3)]
    Ws, infos = api.krr_solve([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
                              [_t(p.y) for p in probs], mode="fcg", inner_maxit=20, max_outer=1000)
    for p, w, i in zip(probs, Ws, infos):
        assert i["status"] == 0
        assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w.cpu().numpy()) <= 1.01e-6
