"""The allocation-free product kmvp_gauss_noalloc (GPU), through the C ABI.

Callers that cannot allocate device memory (graph capture, serving loops) get
the Gaussian product with its scratch in a fixed static device array.  Its
results are held to the workspace entry point kmvp_gauss on the same inputs
(the same kernels and launch shape: equal bit for bit) and to the oracle, on two
calls in a row with the second one smaller (the array keeps the first call's
contents), and a size beyond the array is refused.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import api, native, workloads
from parity import call_vector, check

pytestmark = pytest.mark.gpu


def _noalloc(x, sigma, q, shift, prec):
    lib = native.load()
    pts = native.Points(x.shape[0], x.shape[1], x.data_ptr())
    y = torch.empty_like(q)
    rc = lib.kmvp_gauss_noalloc(ctypes.byref(pts), ctypes.c_double(sigma), ctypes.c_double(shift),
                                ctypes.c_int32(native.PREC[prec]), ctypes.c_void_p(q.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), api._stream())
    return rc, y


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_noalloc_matches_workspace_entry_point(prec):
    lib = native.load()
    lib.kmvp_gauss_noalloc.restype = ctypes.c_int
    lib.krr_noalloc_scratch_bytes.restype = ctypes.c_size_t
    assert lib.krr_noalloc_scratch_bytes() == 128 << 20
    dt = torch.float64 if prec == "fp64" else torch.float32
    # each call smaller than the one before; d = 8 takes the symmetric kernels'
    # d > 3 forms
    for n, d, seed in ((50_000, 3, 1), (8_000, 8, 3), (3_000, 2, 2)):
        if d == 3:
            p = workloads.kriging(n=n)
            xn, sigma, shift = p.x, p.sigma, p.gamma
        elif d == 2:
            p = workloads.plain_small(n=n)
            xn, sigma, shift = p.x, p.sigma, p.gamma
        else:
            xn, sigma, shift = workloads.random_points(40 + seed, n, d, 1.0, kind="normal"), 0.6 * np.sqrt(d), 1e-2
        x = torch.from_numpy(xn).cuda()
        q = torch.from_numpy(workloads.random_vector(40 + seed, n)).to(dt).cuda()
        y_ws = api.kmvp_gauss(x, sigma, q, shift=shift, prec=prec)
        rc, y = _noalloc(x, sigma, q, shift, prec)
        torch.cuda.synchronize()
        assert rc == 0
        assert torch.equal(y, y_ws)
        rows = np.random.default_rng(seed).choice(n, 32, replace=False)
        want = oracle.mvp_rows(xn, sigma, call_vector(q.double().cpu().numpy(), prec), rows, shift=shift)
        check(y.double().cpu().numpy()[rows], want, prec, what=(n, d))


def test_noalloc_refuses_sizes_beyond_its_array():
    lib = native.load()
    lib.kmvp_gauss_noalloc.restype = ctypes.c_int
    n = 400_000
    x = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    q = torch.zeros(n, dtype=torch.float32, device="cuda")
    rc, _ = _noalloc(x, 1.0, q, 0.0, "fp32")
    assert rc == native.KRR_EUNSUPPORTED
