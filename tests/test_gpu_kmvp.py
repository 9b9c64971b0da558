"""Parity of the HIP kernel products with the FP64 oracle (GPU).

Bars (tests/parity.py): FP64 1e-12, FP32 1e-5, BF16-input 1e-2, norm-wise and
element-wise, q ~ N(0, 1).  The oracle evaluates the kernel on the original FP64
points and on the q the call receives (FP32 for the FP32 and BF16 products), so
every rounding inside the library counts against the low precisions.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads
from parity import BAR as TOL, DT, call_vector, check

pytestmark = pytest.mark.gpu


def _api():
    from paper_1408_1237_amd import api
    return api


def _gpu_mvp(x, sigma, q, shift, prec):
    api = _api()
    xt = torch.from_numpy(x).cuda()
    qt = torch.from_numpy(q).to(DT[prec]).cuda()
    y = api.kmvp_gauss(xt, sigma, qt, shift=shift, prec=prec)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 2000])
def test_kmvp_sizes(prec, n):
    x = workloads.random_points(100 + n, n, 3, 2.0)
    q = workloads.random_vector(200 + n, n)
    y = _gpu_mvp(x, 0.6, q, 0.01, prec)
    want = oracle.mvp(x, 0.6, call_vector(q, prec), shift=0.01)
    check(y, want, prec, what=n)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 7, 8, 9, 12, 13, 16, 17, 20, 25, 31, 33, 40, 47, 49, 56, 64])
def test_kmvp_dims(prec, d):
    n = 700
    x = workloads.random_points(300 + d, n, d, 1.0, kind="normal")
    sigma = 0.5 * np.sqrt(d)
    q = workloads.random_vector(400 + d, n)
    y = _gpu_mvp(x, sigma, q, 0.1, prec)
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.1)
    check(y, want, prec, what=d)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_kmvp_coincident_points(prec):
    # K_hat = 1 1^T: y_i = sum(q) + s q_i
    n = 300
    x = np.tile(np.array([[3.0, -2.0, 7.5]]), (n, 1))
    q = workloads.random_vector(5, n)
    y = _gpu_mvp(x, 0.3, q, 0.5, prec)
    qr = q.astype(np.float32).astype(np.float64) if prec != "fp64" else q
    want = qr.sum() + 0.5 * qr
    assert _relerr(y, want) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_kmvp_far_points(prec):
    # points 1000 sigma apart: K_hat = I, y = (1 + s) q (every tile is wide)
    n = 600
    x = np.zeros((n, 2))
    x[:, 0] = np.arange(n) * 1000.0
    q = workloads.random_vector(6, n)
    y = _gpu_mvp(x, 1.0, q, 0.25, prec)
    assert _relerr(y, 1.25 * q) <= TOL[prec]


def test_kmvp_deterministic():
    x = workloads.random_points(7, 5000, 3, 10.0)
    q = workloads.random_vector(8, 5000)
    a = _gpu_mvp(x, 0.5, q, 0.0, "fp32")
    b = _gpu_mvp(x, 0.5, q, 0.0, "fp32")
    assert np.array_equal(a, b)


def test_kmvp_permutation_equivariant():
    x = workloads.random_points(9, 3000, 2, 1.0)
    q = workloads.random_vector(10, 3000)
    perm = np.random.default_rng(11).permutation(3000)
    a = _gpu_mvp(x, 0.1, q, 0.0, "fp64")
    b = _gpu_mvp(np.ascontiguousarray(x[perm]), 0.1, np.ascontiguousarray(q[perm]), 0.0, "fp64")
    assert np.allclose(a[perm], b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kmvp_kriging_shape_sampled_rows(prec):
    # the full kriging shape (N = 1e5, d = 3), checked on 64 sampled rows
    p = workloads.kriging()
    q = workloads.random_vector(7, p.n)
    y = _gpu_mvp(p.x, p.sigma, q, p.gamma, prec)
    rows = np.random.default_rng(12).choice(p.n, 64, replace=False)
    want = oracle.mvp_rows(p.x, p.sigma, call_vector(q, prec), rows, shift=p.gamma)
    check(y[rows], want, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_kmvp_clustered_large_sampled_rows(prec):
    # N = 1e6, d = 2 clustered points (the largest workload: FP64 outer products,
    # BF16-input inner products, FP32 for comparison), 16 sampled rows against
    # the oracle's row sums over all 1e6 sources, with the shift of the inner
    # system (delta) and of the outer one (gamma)
    p = workloads.clustered_large()
    q = workloads.random_vector(7, p.n)
    shift = p.gamma if prec == "fp64" else p.delta
    y = _gpu_mvp(p.x, p.sigma, q, shift, prec)
    rows = np.random.default_rng(13).choice(p.n, 16, replace=False)
    want = oracle.mvp_rows(p.x, p.sigma, call_vector(q, prec), rows, shift=shift)
    check(y[rows], want, prec)


@pytest.mark.parametrize("d,L", [(2, 30.0), (2, 38.0), (2, 41.0), (2, 44.0), (3, 28.0)])
def test_split_f16_worst_case_folded_tiles(d, L):
    # sparse uniform points (sigma = 1, about one neighbour per bandwidth): the
    # 256-point tiles reach squared radii near the fold limit (40 scaled units),
    # where the folded exponent adds its largest terms (|2 t . o| and |c| up to
    # about 2 R^2 and 1.5 R^2) and the split-f16 operands lose the most (2^-22
    # of each); the self pairs dominate every row, so the element-wise bar sees
    # each target's error.  Also targets beyond the tiles' edges, whose exponents
    # against a tile reach the far clamp.
    n = 4096
    x = workloads.random_points(900 + int(L), n, d, L)
    q = workloads.random_vector(901, n)
    y = _gpu_mvp(x, 1.0, q, 0.0, "fp32")
    check(y, oracle.mvp(x, 1.0, call_vector(q, "fp32")), "fp32", what=(d, L))
    ring = workloads.random_points(902, 500, d, 1.0, kind="normal")
    ring = ring / np.linalg.norm(ring, axis=1, keepdims=True) * (0.5 * L * np.sqrt(d) + 8.0) + 0.5 * L
    xt = np.ascontiguousarray(np.concatenate([ring, x[:500]]))
    yc = _gpu_cross(xt, x, 1.0, q, "fp32")
    check(yc, oracle.mvp(xt, 1.0, call_vector(q, "fp32"), xs=x), "fp32", what=(d, L, "cross"))


def _gpu_cross(xt, xs, sigma, q, prec):
    api = _api()
    y = api.kmvp_gauss_cross(torch.from_numpy(xt).cuda(), torch.from_numpy(xs).cuda(), sigma,
                             torch.from_numpy(q).to(DT[prec]).cuda(), prec=prec)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("nt,ns", [(1, 1), (1, 300), (300, 1), (257, 1000), (1000, 257), (3000, 2000)])
def test_kmvp_cross(prec, nt, ns):
    # prediction at new points: y = K_hat(targets, sources) q (eq. GPR_mean, eq. Kriging)
    xs = workloads.random_points(500 + ns, ns, 3, 2.0)
    xt = workloads.random_points(600 + nt, nt, 3, 2.0)
    q = workloads.random_vector(700 + ns, ns)
    y = _gpu_cross(xt, xs, 0.5, q, prec)
    want = oracle.mvp(xt, 0.5, call_vector(q, prec), xs=xs)
    assert y.shape == (nt,)
    check(y, want, prec)


def test_kmvp_cross_equals_square_on_same_points():
    x = workloads.random_points(21, 1500, 2, 1.0)
    q = workloads.random_vector(22, 1500)
    a = _gpu_cross(x, x, 0.1, q, "fp64")
    b = _gpu_mvp(x, 0.1, q, 0.0, "fp64")
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


def test_kmvp_cross_shard_shape_clustered():
    # one shard of a row-sharded product over 8 GPUs at the clustered 1e6 shape:
    # 125,000 target rows x 1,000,000 sources, BF16 inputs, checked on 16 rows
    p = workloads.clustered_large()
    q = workloads.random_vector(7, p.n)
    xt = np.ascontiguousarray(p.x[:125_000])
    y = _gpu_cross(xt, p.x, p.sigma, q, "bf16")
    rows = np.random.default_rng(14).choice(xt.shape[0], 16, replace=False)
    want = oracle.mvp(xt[rows], p.sigma, call_vector(q, "bf16"), xs=p.x)
    check(y[rows], want, "bf16")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 8, 16])
def test_matrix_core_exponent_matches_valu_kernel(monkeypatch, prec, d):
    # products use the matrix-core exponent kernel for d <= 16; KRR_KMVP_VALU=1
    # selects the VALU kernel; both must meet the oracle bar and agree with each
    # other to the precision's rounding
    n = 1500
    x = workloads.random_points(70 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(71 + d, n)
    sigma = 0.6 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    a = _gpu_mvp(x, sigma, q, 0.05, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    b = _gpu_mvp(x, sigma, q, 0.05, prec)
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.05)
    check(a, want, prec)
    check(b, want, prec)
    assert _relerr(a, b) <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,d", [(9000, 3), (20000, 2), (5000, 16), (3000, 20)])
def test_result_independent_of_column_splits(monkeypatch, prec, n, d):
    # partial sums are formed over fixed groups of column tiles, so the product
    # is bitwise the same for every split count the autotuner may pick
    x = workloads.random_points(80 + d, n, d, 3.0)
    q = workloads.random_vector(81 + d, n)
    sigma = 0.5 * np.sqrt(d)
    outs = []
    for k in ("1", "2", "5", "1000"):
        monkeypatch.setenv("KRR_KMVP_SPLITS", k)
        outs.append(_gpu_mvp(x, sigma, q, 0.01, prec))
    monkeypatch.delenv("KRR_KMVP_SPLITS")
    default = _gpu_mvp(x, sigma, q, 0.01, prec)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    if d <= (16 if prec == "fp64" else 12):
        # the default product is the symmetric kernel here: its own fixed
        # summation order and tile anchors (FP64: equal to the exponential's
        # 2.5e-14 per term; FP32 / BF16: to their rounding), the same on every call
        assert _relerr(default, outs[0]) <= (1e-13 if prec == "fp64" else 1e-5)
        assert np.array_equal(default, _gpu_mvp(x, sigma, q, 0.01, prec))
    else:
        assert np.array_equal(default, outs[0])
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.01)
    check(outs[0], want, prec)
    check(default, want, prec)


# The symmetric FP64 product (one exponential per pair for both of its terms)
# against the one-sided kernel (KRR_KMVP_SYM=0) and the oracle: single and
# ragged tiles, one tile per group (up to 100 tiles) and several, every
# compiled dimension up to 16 (d = 16: two row units per tile, one staging
# buffer).
@pytest.mark.parametrize("n,d", [(1, 3), (2, 2), (255, 3), (256, 1), (257, 4), (2000, 2), (2000, 6),
                                 (9000, 3), (26000, 3), (30000, 8), (12000, 12), (40000, 1), (300, 16),
                                 (3000, 16), (27000, 16)])
def test_symmetric_fp64_product(monkeypatch, n, d):
    x = workloads.random_points(500 + d, n, d, 2.0 * d ** 0.5, kind="normal")
    q = workloads.random_vector(501 + d, n)
    sigma = 0.7 * np.sqrt(d)
    monkeypatch.delenv("KRR_KMVP_SYM", raising=False)
    y = _gpu_mvp(x, sigma, q, 0.02, "fp64")
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    y1 = _gpu_mvp(x, sigma, q, 0.02, "fp64")
    monkeypatch.delenv("KRR_KMVP_SYM")
    # each pair's exponential is taken against another tile anchor (the table
    # exponential's 2.5e-14 per term)
    assert _relerr(y, y1) <= 1e-13
    if n <= 12000:
        check(y, oracle.mvp(x, sigma, q, shift=0.02), "fp64", what=(n, d))
    else:
        rows = np.random.default_rng(n).choice(n, 64, replace=False)
        check(y[rows], oracle.mvp_rows(x, sigma, q, rows, shift=0.02), "fp64", what=(n, d))


# The symmetric FP32 / BF16 product (compiled dimensions up to 12, and 16 from
# groups of 8 tiles: N = 200,000) against the one-sided split-f16 kernel and the
# oracle.
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,d", [(1, 1), (200, 2), (257, 3), (3000, 3), (9000, 2), (30000, 1), (26000, 3),
                                 (1, 8), (2, 12), (257, 4), (3000, 5), (9000, 6), (2000, 8), (26000, 8),
                                 (12000, 10), (5000, 12), (30000, 12), (200000, 16)])
def test_symmetric_split_f16_product(monkeypatch, prec, n, d):
    x = workloads.random_points(520 + d, n, d, 2.0 * d ** 0.5, kind="normal")
    q = workloads.random_vector(521 + d, n)
    sigma = 0.7 * np.sqrt(d)
    monkeypatch.delenv("KRR_KMVP_SYM", raising=False)
    y = _gpu_mvp(x, sigma, q, 0.02, prec)
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    y1 = _gpu_mvp(x, sigma, q, 0.02, prec)
    monkeypatch.delenv("KRR_KMVP_SYM")
    assert _relerr(y, y1) <= 1e-5
    qc = call_vector(q, prec)
    if n <= 12000:
        check(y, oracle.mvp(x, sigma, qc, shift=0.02), prec, what=(n, d))
    else:
        rows = np.random.default_rng(n).choice(n, 64, replace=False)
        check(y[rows], oracle.mvp_rows(x, sigma, qc, rows, shift=0.02), prec, what=(n, d))


# The symmetric products keep a column group's source terms in LDS where it fits
# and otherwise add them into the slots in memory; both paths add the same terms
# in the same order (KRR_KMVP_SYM_SLOTS=1 forces the memory path).  At N = 140,000,
# d = 12 (FP64) the groups of 6 tiles exceed the LDS room, so the memory path
# runs either way and is checked against the oracle.
@pytest.mark.parametrize("prec,n,d", [("fp64", 9000, 3), ("fp64", 30000, 12), ("fp64", 27000, 16),
                                      ("fp32", 26000, 3), ("bf16", 9000, 2), ("fp32", 30000, 8),
                                      ("bf16", 12000, 12), ("fp32", 200000, 16), ("fp64", 140000, 12)])
def test_symmetric_slot_paths_agree(monkeypatch, prec, n, d):
    x = workloads.random_points(540 + d, n, d, 2.0 * d ** 0.5, kind="normal")
    q = workloads.random_vector(541 + d, n)
    sigma = 0.7 * np.sqrt(d)
    monkeypatch.delenv("KRR_KMVP_SYM_SLOTS", raising=False)
    y = _gpu_mvp(x, sigma, q, 0.02, prec)
    monkeypatch.setenv("KRR_KMVP_SYM_SLOTS", "1")
    y1 = _gpu_mvp(x, sigma, q, 0.02, prec)
    monkeypatch.delenv("KRR_KMVP_SYM_SLOTS")
    assert np.array_equal(y, y1)
    rows = np.random.default_rng(n + d).choice(n, 48, replace=False)
    qc = call_vector(q, prec)
    check(y[rows], oracle.mvp_rows(x, sigma, qc, rows, shift=0.02), prec, what=(prec, n, d))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_symmetric_fp64_product_wide_tiles(d):
    # 700 points spread over a box hundreds of bandwidths wide: every tile is
    # wider than the FP64 fold limit (direct form in both directions), most
    # pairs underflow, a few neighbours remain
    rng = np.random.default_rng(90 + d)
    x = rng.uniform(0.0, 300.0, size=(700, d))
    x[350:360] = x[349] + rng.normal(0.0, 0.5, size=(10, d))  # a small dense group inside a wide tile
    q = workloads.random_vector(91 + d, 700)
    y = _gpu_mvp(x, 1.0, q, 0.01, "fp64")
    check(y, oracle.mvp(x, 1.0, q, shift=0.01), "fp64", what=d)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 6, 8, 12, 16])
def test_split_f16_kernel_matches_fp32_matrix_kernel(monkeypatch, prec, d):
    # FP32 / BF16 products run the split-f16 matrix-core kernel; KRR_KMVP_MG32=1
    # selects the FP32 matrix-core form; both meet the oracle bar and agree to
    # FP32 rounding (the split keeps the FP32 operands to 2^-22)
    n = 2100
    x = workloads.random_points(90 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(91 + d, n)
    sigma = 0.7 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_MG32", "0")
    a = _gpu_mvp(x, sigma, q, 0.02, prec)
    monkeypatch.setenv("KRR_KMVP_MG32", "1")
    b = _gpu_mvp(x, sigma, q, 0.02, prec)
    monkeypatch.delenv("KRR_KMVP_MG32")
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.02)
    check(a, want, prec)
    check(b, want, prec)
    assert _relerr(a, b) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_split_f16_kernel_far_and_wide_tiles(monkeypatch, prec):
    # three clusters: two tight ones 6 and 40 bandwidths apart (targets of one
    # against tiles of the other: every pair's exponent near or below -200, the
    # clamped case) and a sparse one whose tiles are wide (direct VALU form,
    # offsets beyond the f16 range; also tiles that mix cluster and sparse
    # points, where BF16 offsets would be hundreds of units long and the BF16
    # products keep FP32 offsets).  Both kernel forms meet the oracle bar, on
    # all rows and on the sparse rows alone, and agree with each other.
    rng = np.random.default_rng(17)
    a = rng.normal(0.0, 1.0, size=(1200, 3))
    b = rng.normal(0.0, 1.0, size=(1100, 3)) + np.array([6.0, 0.0, 0.0])
    c = rng.normal(0.0, 1.0, size=(900, 3)) + np.array([0.0, 40.0, 0.0])
    s = rng.uniform(-300.0, 300.0, size=(700, 3)) + np.array([0.0, 0.0, 400.0])
    x = np.ascontiguousarray(np.concatenate([a, b, c, s]))
    q = workloads.random_vector(18, x.shape[0])
    monkeypatch.setenv("KRR_KMVP_MG32", "0")
    y = _gpu_mvp(x, 1.0, q, 0.01, prec)
    monkeypatch.setenv("KRR_KMVP_MG32", "1")
    y_mg = _gpu_mvp(x, 1.0, q, 0.01, prec)
    monkeypatch.delenv("KRR_KMVP_MG32")
    want = oracle.mvp(x, 1.0, call_vector(q, prec), shift=0.01)
    rows = np.arange(3200, 3900)
    for got in (y, y_mg):
        check(got, want, prec)
        check(got[rows], want[rows], prec)
    assert _relerr(y, y_mg) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [6, 12])
def test_symmetric_split_f16_far_and_wide_tiles(monkeypatch, prec, d):
    # the three-cluster set above in d dimensions (clusters 6 and 40 bandwidths
    # apart, a sparse cluster of wide tiles): the symmetric kernel (default for
    # square products up to d = 12) against the one-sided one and the oracle,
    # on all rows and on the sparse rows alone
    rng = np.random.default_rng(19 + d)
    shift_b, shift_c, shift_s = np.zeros(d), np.zeros(d), np.zeros(d)
    shift_b[0], shift_c[1], shift_s[2] = 6.0, 40.0, 400.0
    a = rng.normal(0.0, 1.0, size=(1200, d))
    b = rng.normal(0.0, 1.0, size=(1100, d)) + shift_b
    c = rng.normal(0.0, 1.0, size=(900, d)) + shift_c
    sp = rng.uniform(-300.0, 300.0, size=(700, d)) + shift_s
    x = np.ascontiguousarray(np.concatenate([a, b, c, sp]))
    q = workloads.random_vector(20 + d, x.shape[0])
    sigma = 0.5 * np.sqrt(d)
    monkeypatch.delenv("KRR_KMVP_SYM", raising=False)
    y = _gpu_mvp(x, sigma, q, 0.01, prec)
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    y1 = _gpu_mvp(x, sigma, q, 0.01, prec)
    monkeypatch.delenv("KRR_KMVP_SYM")
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.01)
    rows = np.arange(3200, 3900)
    for got in (y, y1):
        check(got, want, prec, what=d)
        check(got[rows], want[rows], prec, what=d)
    assert _relerr(y, y1) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [17, 24, 29, 32, 41, 48])
def test_split_f16_large_d_matches_valu_kernel(monkeypatch, prec, d):
    # 16 < d <= 48 (compiled at 24, 32, 48): the staged split-f16 kernel meets
    # the oracle bar and agrees with the VALU kernel (KRR_KMVP_VALU=1) to FP32
    # rounding; N = 1300 spans five full column tiles and a ragged one
    n = 1300
    x = workloads.random_points(120 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(121 + d, n)
    sigma = 0.6 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    a = _gpu_mvp(x, sigma, q, 0.03, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    b = _gpu_mvp(x, sigma, q, 0.03, prec)
    monkeypatch.delenv("KRR_KMVP_VALU")
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.03)
    check(a, want, prec)
    check(b, want, prec)
    assert _relerr(a, b) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [24, 48])
def test_split_f16_large_d_far_and_wide_tiles(monkeypatch, prec, d):
    # d-dimensional version of the three-cluster case: two tight clusters 6 and
    # 40 bandwidths apart along different axes (the second pair clamped as far)
    # and a sparse cluster of wide tiles (direct form on FP32 offsets); held to
    # the oracle and to the VALU kernel
    rng = np.random.default_rng(31 + d)
    a = rng.normal(0.0, 0.3, size=(900, d))
    b = rng.normal(0.0, 0.3, size=(800, d))
    b[:, 0] += 6.0
    c = rng.normal(0.0, 0.3, size=(700, d))
    c[:, 1] += 40.0
    s = rng.uniform(-300.0, 300.0, size=(600, d))
    s[:, 2] += 400.0
    x = np.ascontiguousarray(np.concatenate([a, b, c, s]))
    q = workloads.random_vector(32 + d, x.shape[0])
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    y = _gpu_mvp(x, 1.0, q, 0.01, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    y_valu = _gpu_mvp(x, 1.0, q, 0.01, prec)
    monkeypatch.delenv("KRR_KMVP_VALU")
    assert _relerr(y, y_valu) <= 1e-5
    want = oracle.mvp(x, 1.0, call_vector(q, prec), shift=0.01)
    rows = np.arange(2400, 3000)
    check(y, want, prec)
    check(y[rows], want[rows], prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d", [20, 40, 64])
def test_kmvp_cross_large_d(prec, d):
    # prediction at new points through the large-d kernels (staged split-f16 for
    # FP32 / BF16 up to 48, the point-major VALU form otherwise)
    xs = workloads.random_points(800 + d, 1100, d, 1.0, kind="normal")
    xt = workloads.random_points(900 + d, 700, d, 1.0, kind="normal")
    q = workloads.random_vector(1000 + d, 1100)
    sigma = 0.6 * np.sqrt(d)
    y = _gpu_cross(xt, xs, sigma, q, prec)
    want = oracle.mvp(xt, sigma, call_vector(q, prec), xs=xs)
    check(y, want, prec)


@pytest.mark.parametrize("d", [24, 41, 64])
def test_fp64_large_d_far_and_wide_tiles(d):
    # the FP64 VALU product at the large compiled dimensions on the
    # three-cluster set (folded, far and wide tiles) and N(0, I) points
    rng = np.random.default_rng(41 + d)
    a = rng.normal(0.0, 0.3, size=(700, d))
    b = rng.normal(0.0, 0.3, size=(600, d))
    b[:, 0] += 6.0
    c = rng.normal(0.0, 0.3, size=(500, d))
    c[:, 1] += 40.0
    s = rng.uniform(-300.0, 300.0, size=(400, d))
    s[:, 2] += 400.0
    x = np.ascontiguousarray(np.concatenate([a, b, c, s]))
    q = workloads.random_vector(42 + d, x.shape[0])
    y = _gpu_mvp(x, 1.0, q, 0.01, "fp64")
    check(y, oracle.mvp(x, 1.0, q, shift=0.01), "fp64")
    x = workloads.random_points(43 + d, 1100, d, 1.0, kind="normal")
    q = workloads.random_vector(44 + d, 1100)
    sigma = 0.6 * np.sqrt(d)
    y = _gpu_mvp(x, sigma, q, 0.01, "fp64")
    check(y, oracle.mvp(x, sigma, q, shift=0.01), "fp64")


@pytest.mark.parametrize("d", [17, 24, 29, 32, 41, 48, 64])
def test_fp64_matrix_core_large_d_matches_valu_kernel(monkeypatch, d):
    # FP64 products at d > 16 run the staged matrix-core kernel; KRR_KMVP_VALU=1
    # selects the VALU form; both meet the FP64 bar and agree to FP64 rounding
    n = 1300
    x = workloads.random_points(140 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(141 + d, n)
    sigma = 0.6 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    a = _gpu_mvp(x, sigma, q, 0.03, "fp64")
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    b = _gpu_mvp(x, sigma, q, 0.03, "fp64")
    monkeypatch.delenv("KRR_KMVP_VALU")
    want = oracle.mvp(x, sigma, q, shift=0.03)
    check(a, want, "fp64")
    check(b, want, "fp64")
    assert _relerr(a, b) <= 1e-13


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [49, 64])
def test_fp32_matrix_core_d64_matches_valu_kernel(monkeypatch, prec, d):
    # FP32 / BF16 products above d = 48 (compiled at 64) take the staged FP32
    # matrix-core kernel; it meets the oracle bar and agrees with the VALU form
    n = 1300
    x = workloads.random_points(150 + d, n, d, 1.0, kind="normal")
    q = workloads.random_vector(151 + d, n)
    sigma = 0.6 * np.sqrt(d)
    monkeypatch.setenv("KRR_KMVP_VALU", "0")
    a = _gpu_mvp(x, sigma, q, 0.03, prec)
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    b = _gpu_mvp(x, sigma, q, 0.03, prec)
    monkeypatch.delenv("KRR_KMVP_VALU")
    want = oracle.mvp(x, sigma, call_vector(q, prec), shift=0.03)
    check(a, want, prec)
    check(b, want, prec)
    assert _relerr(a, b) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d", [24, 48, 64])
@pytest.mark.parametrize("nt,ns", [(1, 1), (1, 300), (300, 1), (3, 1100)])
def test_kmvp_cross_large_d_tiny_sets(prec, d, nt, ns):
    # single targets or sources through the staged large-d kernels (padded tiles,
    # one ragged stage)
    xs = workloads.random_points(1100 + ns + d, ns, d, 1.0, kind="normal")
    xt = workloads.random_points(1200 + nt + d, nt, d, 1.0, kind="normal")
    q = workloads.random_vector(1300 + ns, ns)
    sigma = 0.6 * np.sqrt(d)
    y = _gpu_cross(xt, xs, sigma, q, prec)
    want = oracle.mvp(xt, sigma, call_vector(q, prec), xs=xs)
    assert y.shape == (nt,)
    check(y, want, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_far_tile_skipping_changes_nothing(monkeypatch, prec):
    # the clustered layout (50 clusters over [0, 100]^2, sigma = 1) at N = 20,000:
    # most tile pairs lie beyond the far threshold and are skipped; their terms
    # are exactly zero, so the product equals the one that computes them
    # (KRR_NO_TILE_SKIP=1) and meets the oracle bar; the profile reports the
    # skipped share
    from paper_1408_1237_amd import native
    p = workloads.clustered_large(n=20_000)
    q = workloads.random_vector(71, p.n)
    monkeypatch.setenv("KRR_NO_TILE_SKIP", "0")
    with native.profile() as prof:
        y = _gpu_mvp(p.x, p.sigma, q, p.delta, prec)
    monkeypatch.setenv("KRR_NO_TILE_SKIP", "1")
    with native.profile() as prof_all:
        y_all = _gpu_mvp(p.x, p.sigma, q, p.delta, prec)
    monkeypatch.delenv("KRR_NO_TILE_SKIP")
    assert np.array_equal(y, y_all)
    check(y, oracle.mvp(p.x, p.sigma, call_vector(q, prec), shift=p.delta), prec)
    st = prof.stats[prec]
    lo = 0.1 if prec == "fp64" else 0.4  # FP64 skips only beyond exponent -1100, FP32 / BF16 beyond -200
    assert st["launches"] == 1 and lo * st["pairs"] < st["pairs_skipped"] < st["pairs"]
    assert prof_all.stats[prec]["pairs_skipped"] == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_far_tile_skipping_cross_product(monkeypatch, prec):
    # targets in a cluster 60 bandwidths from every source (all their tile pairs
    # skipped: exactly zero) next to targets inside the sources' cluster
    xs = workloads.random_points(72, 3000, 2, 1.0, kind="normal")
    far = workloads.random_points(73, 700, 2, 1.0, kind="normal") + np.array([60.0, 0.0])
    near = workloads.random_points(74, 300, 2, 1.0, kind="normal")
    xt = np.ascontiguousarray(np.concatenate([far, near]))
    q = workloads.random_vector(75, 3000)
    y = _gpu_cross(xt, xs, 1.0, q, prec)
    assert np.all(y[:700] == 0.0)
    check(y, oracle.mvp(xt, 1.0, call_vector(q, prec), xs=xs), prec)
    monkeypatch.setenv("KRR_NO_TILE_SKIP", "1")
    y_all = _gpu_cross(xt, xs, 1.0, q, prec)
    monkeypatch.delenv("KRR_NO_TILE_SKIP")
    assert np.array_equal(y, y_all)
