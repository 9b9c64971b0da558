"""The Matern-3/2 kernel (eq. MaternKernel, section 6) on the GPU.

Products in every precision against the oracle's on-the-fly FP64 sum at the bars
of tests/parity.py (FP64 1e-12, FP32 1e-5, BF16-input 1e-2, norm-wise and
element-wise, the oracle on the q the call receives), special cases, and solves
(flexible GMRES, plain FP64 CG, several systems) against the oracle's Cholesky
solve with the explicit Matern matrix.  The Matern kernel is flat near zero
distance, so at larger d many comparable terms of both signs enter every row
sum; there the BF16 rounding of q alone moves the exact product by about 1e-2,
and the BF16 bar is 1.25 times that format floor (parity.format_floor: the
oracle on the BF16-rounded q against the oracle on q).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads
from parity import BAR as TOL, DT, call_vector, check, format_floor

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mvp(x, h, q, shift, prec):
    from paper_1408_1237_amd import api
    y = api.kmvp_matern(_t(x), h, _t(q).to(DT[prec]), shift=shift, prec=prec)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,d", [(1, 2), (257, 1), (2000, 2), (1500, 3), (3000, 8), (700, 17), (900, 40),
                                 (600, 64)])
def test_matern_product_matches_oracle(prec, n, d):
    x = workloads.random_points(100 + n + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(101 + n, n)
    h = 0.7 * np.sqrt(d)
    ref = lambda v: oracle.matern_mvp(x, h, v, shift=0.05)  # noqa: E731
    q32 = call_vector(q, prec)
    floor = format_floor(ref, q32) if prec == "bf16" else (0.0, 0.0)
    check(_mvp(x, h, q, 0.05, prec), ref(q32), prec, floor=floor, what=(n, d))


def test_matern_special_cases_and_kernel_selection():
    from paper_1408_1237_amd import api
    q = workloads.random_vector(110, 300)
    y = _mvp(np.zeros((300, 3)), 1.0, q, 0.5, "fp64")       # coincident: K_hat = 1 1^T
    assert np.allclose(y, q.sum() + 0.5 * q, rtol=1e-12)
    far = np.arange(300, dtype=float).reshape(-1, 1) * 100.0  # far apart: K_hat = I
    assert np.allclose(_mvp(far, 1.0, q, 0.0, "fp64"), q, rtol=1e-14)
    x = workloads.random_points(111, 500, 2, 1.0)
    qt = _t(workloads.random_vector(112, 500))
    g = api.kmvp_gauss(_t(x), 0.3, qt, prec="fp64").cpu().numpy()
    m = api.kmvp_matern(_t(x), 0.3, qt, prec="fp64").cpu().numpy()
    assert _rel(m, g) > 1e-2  # two different kernels


def test_matern_sampled_rows_at_1e5():
    p = workloads.matern_classification(n=100_000)
    q = workloads.random_vector(113, p.n)
    for prec in ("fp64", "fp32"):
        y = _mvp(p.x, p.sigma, q, p.gamma, prec)
        rows = np.random.default_rng(7).choice(p.n, 48, replace=False)
        want = oracle.matern_mvp_rows(p.x, p.sigma, call_vector(q, prec), rows, shift=p.gamma)
        check(y[rows], want, prec)


@pytest.mark.parametrize("inner_prec", ["fp32", "bf16"])
def test_matern_fgmres_matches_direct_solve(inner_prec):
    from paper_1408_1237_amd import api
    p = workloads.matern_classification(n=1500, d=5)
    w, info = api.fgmres_solve(_t(p.x), p.sigma, p.gamma, _t(p.y), kernel="matern32", inner_prec=inner_prec,
                               inner_maxit=20, restart_m=50, max_outer=500)
    assert info["status"] == 0 and info["relres_true"] <= 1e-6
    wn = w.cpu().numpy()
    r = p.y - oracle.matern_mvp(p.x, p.sigma, wn, shift=p.gamma)
    assert np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(p.y)
    ws = oracle.matern_direct_solve(p.x, p.sigma, p.gamma, p.y)
    K = oracle.matern_matrix(p.x, p.sigma) + p.gamma * np.eye(p.n)
    kappa = np.linalg.cond(K)
    assert np.linalg.norm(wn - ws) <= 2 * kappa * 1e-6 * np.linalg.norm(ws)


def test_matern_cg64_and_several_systems():
    from paper_1408_1237_amd import api
    probs = [workloads.matern_classification(seed=120 + k, n=800 + 300 * k, d=4) for k in range(3)]
    Ws, infos = api.krr_solve([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
                              [_t(p.y) for p in probs], mode="fgmres", kernel="matern32", inner_maxit=20,
                              restart_m=50, max_outer=500)
    for p, w, i in zip(probs, Ws, infos):
        assert i["status"] == 0
        r = p.y - oracle.matern_mvp(p.x, p.sigma, w.cpu().numpy(), shift=p.gamma)
        assert np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(p.y)
    (w64,), (i64,) = api.krr_solve([_t(probs[1].x)], [probs[1].sigma], [probs[1].gamma], [_t(probs[1].y)],
                                   mode="cg64", kernel="matern32", max_outer=20000)
    assert i64["status"] == 0
    r = probs[1].y - oracle.matern_mvp(probs[1].x, probs[1].sigma, w64.cpu().numpy(), shift=probs[1].gamma)
    assert np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(probs[1].y)


def test_matern_unknown_kernel_rejected():
    from paper_1408_1237_amd import api, native
    p = workloads.matern_classification(n=200, d=2)
    with pytest.raises(native.KrrError):
        api.fgmres_solve(_t(p.x), p.sigma, p.gamma, _t(p.y), kernel=7)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 6, 8, 12, 16, 17, 24, 33, 48])
def test_matern_matrix_core_kernel_matches_valu_kernel(monkeypatch, prec, d):
    # FP32 / BF16 Matern products at d <= 48 form the squared distance on the
    # matrix cores (split-f16; staged sources above 16); KRR_KMVP_VALU=1 selects
    # the VALU kernel.  The two agree to FP32 rounding on the same rounded
    # inputs, and both meet the oracle bar (BF16: or its format floor, see the
    # module docstring)
    n = 1900
    x = workloads.random_points(120 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(121 + d, n)
    h = 0.8 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    a = _mvp(x, h, q, 0.03, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    b = _mvp(x, h, q, 0.03, prec)
    monkeypatch.delenv("KRR_KMVP_VALU")
    ref = lambda v: oracle.matern_mvp(x, h, v, shift=0.03)  # noqa: E731
    q32 = call_vector(q, prec)
    want = ref(q32)
    floor = format_floor(ref, q32) if prec == "bf16" else (0.0, 0.0)
    assert _rel(a, b) <= 1e-5
    check(a, want, prec, floor=floor)
    check(b, want, prec, floor=floor)


# The symmetric Matern product (square products up to d = 16 in every precision;
# one kernel value per unordered pair for both of its terms) against the
# one-sided kernel (KRR_KMVP_SYM=0) and the oracle: a single point, ragged
# tiles, one and several tiles per group.
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,d", [(1, 3), (300, 1), (2500, 3), (9000, 8), (4000, 12), (30000, 2), (20000, 16),
                                 (200000, 16)])
def test_matern_symmetric_product(monkeypatch, prec, n, d):
    x = workloads.random_points(140 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(141 + d, n)
    h = 0.8 * np.sqrt(d)
    monkeypatch.delenv("KRR_KMVP_SYM", raising=False)
    y = _mvp(x, h, q, 0.03, prec)
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    y1 = _mvp(x, h, q, 0.03, prec)
    monkeypatch.delenv("KRR_KMVP_SYM")
    assert _rel(y, y1) <= (1e-12 if prec == "fp64" else 1e-5)
    q32 = call_vector(q, prec)
    rows = np.arange(n) if n <= 9000 else np.random.default_rng(n).choice(n, 64, replace=False)
    ref = lambda v: oracle.matern_mvp_rows(x, h, v, rows, shift=0.03)  # noqa: E731
    floor = format_floor(ref, q32) if prec == "bf16" else (0.0, 0.0)
    check(y[rows], ref(q32), prec, floor=floor, what=(n, d))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_matern_matrix_core_kernel_far_and_wide_tiles(monkeypatch, prec):
    # two tight clusters 150 length scales apart (targets of one are beyond the
    # clamp distance from every tile of the other) and a sparse cluster with wide
    # tiles; the default (symmetric) product is held to the oracle (all rows and
    # the sparse rows; BF16: or its format floor) and to the VALU kernel
    rng = np.random.default_rng(23)
    a = rng.normal(0.0, 1.0, size=(1000, 2))
    b = rng.normal(0.0, 1.0, size=(900, 2)) + np.array([150.0, 0.0])
    s = rng.uniform(-3000.0, 3000.0, size=(500, 2)) + np.array([0.0, 5000.0])
    x = np.ascontiguousarray(np.concatenate([a, b, s]))
    q = workloads.random_vector(24, x.shape[0])
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    y = _mvp(x, 1.0, q, 0.01, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    yv = _mvp(x, 1.0, q, 0.01, prec)
    monkeypatch.delenv("KRR_KMVP_VALU")
    q32 = call_vector(q, prec)
    ref = lambda v: oracle.matern_mvp(x, 1.0, v, shift=0.01)  # noqa: E731
    want = ref(q32)
    assert _rel(y, yv) <= 1e-5
    rows = np.arange(1900, 2400)
    if prec == "bf16":
        check(y, want, prec, floor=format_floor(ref, q32))
        rref = lambda v: ref(v)[rows]  # noqa: E731
        check(y[rows], want[rows], prec, floor=format_floor(rref, q32))
    else:
        check(y, want, prec)
        check(y[rows], want[rows], prec)


@pytest.mark.parametrize("d", [24, 48])
def test_matern_matrix_core_large_d_far_and_wide_tiles(monkeypatch, d):
    # the same three-cluster construction in d dimensions for the staged kernel
    rng = np.random.default_rng(25 + d)
    a = rng.normal(0.0, 0.3, size=(900, d))
    b = rng.normal(0.0, 0.3, size=(800, d))
    b[:, 0] += 150.0
    s = rng.uniform(-3000.0, 3000.0, size=(500, d))
    s[:, 1] += 5000.0
    x = np.ascontiguousarray(np.concatenate([a, b, s]))
    q = workloads.random_vector(26 + d, x.shape[0])
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    y = _mvp(x, 1.0, q, 0.01, "fp32")
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    yv = _mvp(x, 1.0, q, 0.01, "fp32")
    monkeypatch.delenv("KRR_KMVP_VALU")
    want = oracle.matern_mvp(x, 1.0, call_vector(q, "fp32"), shift=0.01)
    assert _rel(y, yv) <= 1e-5
    check(y, want, "fp32")
    rows = np.arange(1700, 2200)
    check(y[rows], want[rows], "fp32")


@pytest.mark.parametrize("prec,d", [("fp64", 1), ("fp64", 2), ("fp64", 3), ("fp64", 4), ("fp64", 6), ("fp64", 8),
                                    ("fp64", 12), ("fp64", 16), ("fp64", 24), ("fp64", 41), ("fp64", 64),
                                    ("fp32", 56), ("fp32", 64), ("bf16", 64)])
def test_matern_staged_matrix_core_matches_valu_kernel(monkeypatch, prec, d):
    # FP64 Matern products (and FP32 / BF16 ones above d = 48, with the source
    # constant formed from the staged offsets) form (log2(e) s)^2 on the matrix
    # cores from [o, 1, |o'|^2] .
    # [-2 log2(e)^2 t, |t'|^2, 1]; they meet the oracle bar and agree with the
    # VALU form
    n = 1300
    x = workloads.random_points(180 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(181 + d, n)
    h = 0.8 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    a = _mvp(x, h, q, 0.03, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    b = _mvp(x, h, q, 0.03, prec)
    monkeypatch.delenv("KRR_KMVP_VALU")
    ref = lambda v: oracle.matern_mvp(x, h, v, shift=0.03)  # noqa: E731
    q32 = call_vector(q, prec)
    want = ref(q32)
    floor = format_floor(ref, q32) if prec == "bf16" else (0.0, 0.0)
    check(a, want, prec, floor=floor)
    check(b, want, prec, floor=floor)
    assert _rel(a, b) <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("d", [2, 8, 24])
def test_matern_fp64_matrix_core_far_and_wide_tiles(d):
    # FP64 Matern products on the three-cluster set (folded, far and wide tiles)
    rng = np.random.default_rng(27 + d)
    a = rng.normal(0.0, 0.3, size=(700, d))
    b = rng.normal(0.0, 0.3, size=(600, d))
    b[:, 0] += 150.0
    s = rng.uniform(-3000.0, 3000.0, size=(400, d))
    s[:, 1] += 5000.0
    x = np.ascontiguousarray(np.concatenate([a, b, s]))
    q = workloads.random_vector(28 + d, x.shape[0])
    y = _mvp(x, 1.0, q, 0.01, "fp64")
    check(y, oracle.matern_mvp(x, 1.0, q, shift=0.01), "fp64")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d", [5, 7, 13, 20, 31, 47, 49, 56])
def test_matern_product_dims(prec, d):
    # dimensions between the compiled ones (padded) through every Matern kernel
    n = 700
    x = workloads.random_points(190 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(191 + d, n)
    h = 0.7 * np.sqrt(d)
    ref = lambda v: oracle.matern_mvp(x, h, v, shift=0.05)  # noqa: E731
    q32 = call_vector(q, prec)
    floor = format_floor(ref, q32) if prec == "bf16" else (0.0, 0.0)
    check(_mvp(x, h, q, 0.05, prec), ref(q32), prec, floor=floor, what=d)
