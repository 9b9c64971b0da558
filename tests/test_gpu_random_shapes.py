"""Seeded random shapes through every product kernel (GPU): point count, dimension,
precision, kernel family and square / cross form drawn per case, each result
held to the oracle at its precision's bar (FP64 1e-12, FP32 1e-5, BF16 inputs
2e-2 norm-wise)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads

pytestmark = pytest.mark.gpu

BAR = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 2e-2}
DT = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.float32}


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
    if kind == "gauss":
        y = api.kmvp_gauss(xt, h, qt, shift=0.02, prec=prec)
        want = oracle.mvp(x, h, q, shift=0.02)
    else:
        y = api.kmvp_matern(xt, h, qt, shift=0.02, prec=prec)
        want = oracle.matern_mvp(x, h, q, shift=0.02)
    torch.cuda.synchronize()
    y = y.double().cpu().numpy()
    err = np.linalg.norm(y - want) / max(np.linalg.norm(want), 1e-300)
    assert err <= BAR[prec], (n, d, prec, kind, err)


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
    want = oracle.mvp(xt, h, q, xs=xs)
    err = np.linalg.norm(y - want) / max(np.linalg.norm(want), 1e-300)
    assert y.shape == (nt,) and err <= BAR[prec], (nt, n, d, prec, err)
