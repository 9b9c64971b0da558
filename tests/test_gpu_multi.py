"""Parity of the matrix-core multi-RHS product with the FP64 oracle (GPU).

Y = K_hat Q + shift Q for column-major Q (n x nrhs).  Every column is held to the
bars of the single product (tests/parity.py: FP64 1e-12, FP32 1e-5, BF16 inputs
1e-2, norm-wise and element-wise) against the oracle on the Q the call receives
(FP32 for FP32 and BF16 products).  Where the BF16 rounding of a column alone
moves its exact product by more than 1e-2 (smooth kernels on dense sets), that
column's BF16 bar is 1.25 times the format floor, computed with the oracle alone.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads
from parity import BAR as TOL, DT, call_vector, check, format_floor

pytestmark = pytest.mark.gpu


def _gpu_multi(x, sigma, Q, shift, prec):
    from paper_1408_1237_amd import api
    Qt = torch.from_numpy(np.ascontiguousarray(Q.T)).to(DT[prec]).cuda().t()
    Y = api.kmvp_gauss_multi(torch.from_numpy(x).cuda(), sigma, Qt, shift=shift, prec=prec)
    torch.cuda.synchronize()
    return Y.double().cpu().numpy()


def _check_cols(Y, x, sigma, Q, shift, prec):
    """Every column against the oracle (with its BF16 format floor)."""
    Q32 = call_vector(Q, prec)
    W = oracle.mvp_multi(x, sigma, Q32, shift=shift)
    for r in range(Q.shape[1]):
        floor = (0.0, 0.0)
        if prec == "bf16":
            floor = format_floor(lambda v: oracle.mvp(x, sigma, v, shift=shift), np.ascontiguousarray(Q32[:, r]))
        check(Y[:, r], W[:, r], prec, floor=floor, what=r)
    return W


def _colerr(Y, W):
    return max(np.linalg.norm(Y[:, r] - W[:, r]) / max(np.linalg.norm(W[:, r]), 1e-300) for r in range(W.shape[1]))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (5, 16), (300, 3), (1000, 16), (1000, 17), (2049, 33)])
def test_multi_sizes(prec, n, nrhs):
    x = workloads.random_points(800 + n, n, 3, 2.0)
    Q = workloads.random_vector(900 + n, n, nrhs)
    Y = _gpu_multi(x, 0.6, Q, 0.05, prec)
    assert Y.shape == (n, nrhs)
    _check_cols(Y, x, 0.6, Q, 0.05, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 2, 4, 8, 16, 24, 40])
def test_multi_dims(prec, d):
    n = 600
    x = workloads.random_points(1000 + d, n, d, 1.0, kind="normal")
    sigma = np.sqrt(d)
    Q = workloads.random_vector(1100 + d, n, 16)
    Y = _gpu_multi(x, sigma, Q, 0.01, prec)
    _check_cols(Y, x, sigma, Q, 0.01, prec)


def test_multi_far_points_identity():
    # every tile wide: the direct path; K_hat = I
    n = 700
    x = np.zeros((n, 2))
    x[:, 1] = np.arange(n) * 500.0
    Q = workloads.random_vector(12, n, 16)
    for prec in ("fp64", "fp32"):
        Y = _gpu_multi(x, 1.0, Q, 0.5, prec)
        for r in range(16):
            check(Y[:, r], 1.5 * call_vector(Q[:, r], prec), prec)


def test_multi_matches_single_products():
    from paper_1408_1237_amd import api
    x = workloads.random_points(13, 3000, 4, 1.0, kind="normal")
    Q = workloads.random_vector(14, 3000, 16)
    Y = _gpu_multi(x, 2.0, Q, 0.1, "fp64")
    xt = torch.from_numpy(x).cuda()
    for r in (0, 7, 15):
        y = api.kmvp_gauss(xt, 2.0, torch.from_numpy(np.ascontiguousarray(Q[:, r])).cuda(), shift=0.1, prec="fp64")
        assert np.allclose(Y[:, r], y.cpu().numpy(), rtol=1e-12, atol=1e-12 * np.abs(y.cpu().numpy()).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_batched_shape_sampled_rows(prec):
    # the largest batched system shape: N = 50,000, d = 8, 16 right-hand sides, sampled rows
    rng = np.random.default_rng(15)
    n = 50_000
    x = np.ascontiguousarray(rng.standard_normal((n, 8)))
    Q = np.asfortranarray(rng.standard_normal((n, 16)))
    Y = _gpu_multi(x, np.sqrt(8.0), Q, 0.1, prec)
    rows = rng.choice(n, 24, replace=False)
    for r in (0, 9, 15):
        want = oracle.mvp_rows(x, np.sqrt(8.0), call_vector(np.ascontiguousarray(Q[:, r]), prec), rows, shift=0.1)
        check(Y[rows, r], want, prec)


def test_multi_gp_regression_shape_sampled_rows():
    # d = 16 at the GP-regression shape (N = 2e5), 16 right-hand sides, FP32, sampled rows
    p = workloads.gp_regression()
    Q = workloads.random_vector(16, p.n, 16)
    Y = _gpu_multi(p.x, p.sigma, Q, 0.0, "fp32")
    rows = np.random.default_rng(17).choice(p.n, 8, replace=False)
    for r in (0, 15):
        want = oracle.mvp_rows(p.x, p.sigma, call_vector(np.ascontiguousarray(Q[:, r]), "fp32"), rows)
        check(Y[rows, r], want, "fp32")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 6, 8, 12, 16])
def test_multi_split_exponent_matches_valu_exponent(monkeypatch, prec, d):
    # FP32 / BF16 multi-RHS products at d <= 16 form the kernel values on the
    # matrix cores (split-f16 exponent); KRR_KMVP_MULTI_VALU=1 forms them on the
    # VALU; both meet the oracle bar and agree to FP32 rounding
    n = 1300
    x = workloads.random_points(130 + d, n, d, 1.0, kind="normal")
    Q = workloads.random_vector(131 + d, n, 16)
    sigma = 0.7 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_MULTI_VALU", "0")
    A = _gpu_multi(x, sigma, Q, 0.02, prec)
    monkeypatch.setenv("KRR_KMVP_MULTI_VALU", "1")
    B = _gpu_multi(x, sigma, Q, 0.02, prec)
    monkeypatch.delenv("KRR_KMVP_MULTI_VALU")
    _check_cols(A, x, sigma, Q, 0.02, prec)
    _check_cols(B, x, sigma, Q, 0.02, prec)
    assert _colerr(A, B) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_multi_split_exponent_far_and_wide_tiles(monkeypatch, prec):
    # tight clusters far apart (clamped targets) and a sparse cluster (wide
    # tiles, and tiles mixing cluster and sparse points, which keep FP32 offsets
    # in BF16 products); both exponent forms against the oracle on every column,
    # on the sparse rows alone, and against each other
    rng = np.random.default_rng(31)
    a = rng.normal(0.0, 1.0, size=(900, 3))
    b = rng.normal(0.0, 1.0, size=(800, 3)) + np.array([40.0, 0.0, 0.0])
    s = rng.uniform(-300.0, 300.0, size=(500, 3)) + np.array([0.0, 0.0, 400.0])
    x = np.ascontiguousarray(np.concatenate([a, b, s]))
    Q = workloads.random_vector(32, x.shape[0], 16)
    monkeypatch.setenv("KRR_KMVP_MULTI_VALU", "0")
    Y = _gpu_multi(x, 2.0, Q, 0.01, prec)
    monkeypatch.setenv("KRR_KMVP_MULTI_VALU", "1")
    B = _gpu_multi(x, 2.0, Q, 0.01, prec)
    monkeypatch.delenv("KRR_KMVP_MULTI_VALU")
    assert _colerr(Y, B) <= 1e-5
    W = _check_cols(Y, x, 2.0, Q, 0.01, prec)
    rows = np.arange(1700, 2200)
    for r in range(16):
        check(Y[rows, r], W[rows, r], prec, what=r)
