"""Seeded random shapes through every product kernel (GPU): point count, dimension,
precision, kernel family and square / cross form drawn per case, each result
held to the oracle at its precision's bar, norm-wise and element-wise
(tests/parity.py: FP64 1e-12, FP32 1e-5, BF16 inputs 1e-2).  The Matern-3/2
kernel is flat near zero distance, so at large d many comparable terms of both
signs enter every row; there the BF16 rounding of q alone can move the exact
product by more than 1e-2, and its BF16 bar is 1.25 times that format floor (the
oracle on the BF16-rounded q against the oracle on q)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads
from parity import DT, call_vector, check, format_floor

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.choice([1, 2, 17, 255, 256, 257, int(rng.integers(3, 2600))]))
    d = int(rng.integers(1, 65))
    prec = str(rng.choice(["fp64", "fp32", "bf16"]))
    kind = str(rng.choice(["gauss", "matern"]))
    return n, d, prec, kind


@pytest.mark.parametrize("seed", range(24))
def test_random_shape_square_product(seed):
    from paper_1408_1237_amd import api
    n, d, prec, kind = _case(seed)
    x = workloads.random_points(6000 + seed, n, d, 1.0, kind="normal")
    q = workloads.random_vector(6100 + seed, n)
    h = 0.7 * np.sqrt(d)
    xt, qt = torch.from_numpy(x).cuda(), torch.from_numpy(q).to(DT[prec]).cuda()
    q32 = call_vector(q, prec)
    if kind == "gauss":
        y = api.kmvp_gauss(xt, h, qt, shift=0.02, prec=prec)
        ref = lambda v: oracle.mvp(x, h, v, shift=0.02)  # noqa: E731
    else:
        y = api.kmvp_matern(xt, h, qt, shift=0.02, prec=prec)
        ref = lambda v: oracle.matern_mvp(x, h, v, shift=0.02)  # noqa: E731
    torch.cuda.synchronize()
    floor = format_floor(ref, q32) if (prec == "bf16" and kind == "matern") else (0.0, 0.0)
    check(y.double().cpu().numpy(), ref(q32), prec, floor=floor, what=(n, d, kind))


@pytest.mark.parametrize("seed", range(12))
def test_random_shape_cross_product(seed):
    from paper_1408_1237_amd import api
    n, d, prec, _ = _case(100 + seed)
    nt = int(np.random.default_rng(7000 + seed).integers(1, 900))
    xs = workloads.random_points(7100 + seed, n, d, 1.0, kind="normal")
    xt = workloads.random_points(7200 + seed, nt, d, 1.0, kind="normal")
    q = workloads.random_vector(7300 + seed, n)
    h = 0.7 * np.sqrt(d)
    y = api.kmvp_gauss_cross(torch.from_numpy(xt).cuda(), torch.from_numpy(xs).cuda(), h,
                             torch.from_numpy(q).to(DT[prec]).cuda(), prec=prec)
    torch.cuda.synchronize()
    y = y.double().cpu().numpy()
    want = oracle.mvp(xt, h, call_vector(q, prec), xs=xs)
    assert y.shape == (nt,)
    check(y, want, prec, what=(nt, n, d))
