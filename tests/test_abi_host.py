"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, sizes workspaces and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1408_1237_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "krr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|size_t|void|const char\s*\*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_calls():
    assert set(_declared()) == set(N.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = N.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults():
    assert N.status_string(0) == "KRR_OK"
    assert "workspace" in N.status_string(N.KRR_EWORKSPACE)
    o = N.default_opts()
    # the paper's rules (section 6): outer tol 1e-6; delta and inner tol derived at call time
    assert o.tol == 1e-6 and o.delta < 0 and o.inner_tol < 0
    assert o.restart_m == 30 and o.inner_maxit == 10 and o.inner_prec == N.KRR_FP32


def test_workspace_sizes_scale_and_reject_bad_shapes():
    a = N.workspace_size(N.KRR_WS_KMVP, [(1000, 3)])
    b = N.workspace_size(N.KRR_WS_KMVP, [(100000, 3)])
    assert 0 < a < b
    f = N.workspace_size(N.KRR_WS_FGMRES, [(100000, 3)])
    # V (m+1) and Z (m) columns of FP64 dominate the flexible solver
    assert f >= 61 * 100096 * 8
    assert N.workspace_size(N.KRR_WS_KMVP, [(0, 3)]) == 0
    assert N.workspace_size(N.KRR_WS_KMVP, [(10, 0)]) == 0
    assert N.workspace_size(N.KRR_WS_KMVP, [(10, N.KRR_MAX_DIM + 1)]) == 0
    assert N.workspace_size(N.KRR_WS_SOLVE, [(10, 2), (20, 3)], nrhs=0) == 0
    bad = N.default_opts()
    bad.restart_m = 0
    assert N.workspace_size(N.KRR_WS_FGMRES, [(100, 2)], opts=bad) == 0


def test_invalid_arguments_rejected_before_any_launch():
    lib = N.load()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    p = N.Points(10, 2, fake.value)
    ws = ctypes.c_void_p(0x2000)
    # sigma <= 0, bad precision, null vectors, aliasing, d out of range
    assert lib.kmvp_gauss(ctypes.byref(p), 0.0, 0.0, 0, fake, ctypes.c_void_p(0x3000), ws, 1 << 30, None) == N.KRR_EINVAL
    assert lib.kmvp_gauss(ctypes.byref(p), 1.0, 0.0, 7, fake, ctypes.c_void_p(0x3000), ws, 1 << 30, None) == N.KRR_EINVAL
    assert lib.kmvp_gauss(ctypes.byref(p), 1.0, 0.0, 0, None, ctypes.c_void_p(0x3000), ws, 1 << 30, None) == N.KRR_EINVAL
    assert lib.kmvp_gauss(ctypes.byref(p), 1.0, 0.0, 0, fake, fake, ws, 1 << 30, None) == N.KRR_EINVAL
    assert lib.kmvp_gauss(ctypes.byref(p), float("nan"), 0.0, 0, fake, ctypes.c_void_p(0x3000), ws, 1 << 30, None) == N.KRR_EINVAL
    p_bad = N.Points(10, N.KRR_MAX_DIM + 1, fake.value)
    assert lib.kmvp_gauss(ctypes.byref(p_bad), 1.0, 0.0, 0, fake, ctypes.c_void_p(0x3000), ws, 1 << 30, None) == N.KRR_EINVAL
    p0 = N.Points(0, 2, fake.value)
    assert lib.kmvp_gauss(ctypes.byref(p0), 1.0, 0.0, 0, fake, ctypes.c_void_p(0x3000), ws, 1 << 30, None) == N.KRR_EINVAL
    # workspace missing or too small
    assert lib.kmvp_gauss(ctypes.byref(p), 1.0, 0.0, 0, fake, ctypes.c_void_p(0x3000), None, 0, None) == N.KRR_EWORKSPACE
    assert lib.kmvp_gauss(ctypes.byref(p), 1.0, 0.0, 0, fake, ctypes.c_void_p(0x3000), ws, 16, None) == N.KRR_EWORKSPACE
    # solver options: gamma < 0, restart 0, inner maxit 0 with the CG inner solve
    info = N.Info()
    assert lib.fgmres_solve(ctypes.byref(p), 1.0, -1.0, fake, ctypes.c_void_p(0x3000), None, ctypes.byref(info),
                            ws, 1 << 30, None) == N.KRR_EINVAL
    o = N.default_opts()
    o.restart_m = 0
    assert lib.fgmres_solve(ctypes.byref(p), 1.0, 0.1, fake, ctypes.c_void_p(0x3000), ctypes.byref(o),
                            ctypes.byref(info), ws, 1 << 30, None) == N.KRR_EINVAL
    o = N.default_opts()
    o.inner_maxit = 0
    assert lib.fgmres_solve(ctypes.byref(p), 1.0, 0.1, fake, ctypes.c_void_p(0x3000), ctypes.byref(o),
                            ctypes.byref(info), ws, 1 << 30, None) == N.KRR_EINVAL
    assert lib.cg_inner_solve(ctypes.byref(p), 1.0, 0.1, 1, fake, ctypes.c_void_p(0x3000), 0, 0.0, None,
                              ws, 1 << 30, None) == N.KRR_EINVAL
    # krr_solve: bad mode, nrhs 0
    sig = (ctypes.c_double * 1)(1.0)
    gam = (ctypes.c_double * 1)(0.1)
    yp = (ctypes.c_void_p * 1)(fake.value)
    wp = (ctypes.c_void_p * 1)(0x3000)
    assert lib.krr_solve(ctypes.byref(p), 1, sig, gam, 1, yp, None, wp, 9, None, None, ws, 1 << 30, None) == N.KRR_EINVAL
    assert lib.krr_solve(ctypes.byref(p), 1, sig, gam, 0, yp, None, wp, 0, None, None, ws, 1 << 30, None) == N.KRR_EINVAL


def test_probe_rejects_bad_arguments_on_the_host():
    lib = N.load()
    assert lib.krr_probe_workspace_size() > 0
    rates = (ctypes.c_double * 6)()
    assert lib.krr_probe_issue_rates(rates, None, 0, None) == N.KRR_EWORKSPACE
    assert lib.krr_probe_issue_rates(None, None, 0, None) == N.KRR_EINVAL


def _textbook_cg_coefficients(A, b, k):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    alpha, beta = [], []
    for _ in range(k):
        Ap = A @ p
        a = rr / (p @ Ap)
        x += a * p
        r -= a * Ap
        rr_new = r @ r
        alpha.append(a)
        beta.append(rr_new / rr)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return np.array(alpha), np.array(beta)


def test_lanczos_extremes_recover_the_spectrum():
    # host-only computation: after n steps of CG on an n x n SPD matrix the
    # Lanczos tridiagonal has the matrix's eigenvalues; after one step its only
    # Ritz value is the Rayleigh quotient of the right-hand side
    from paper_1408_1237_amd import api
    rng = np.random.default_rng(4)
    n = 24
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.linspace(0.5, 20.0, n)
    A = (Q * ev) @ Q.T
    b = rng.standard_normal(n)
    al, be = _textbook_cg_coefficients(A, b, n)
    lo, hi = api.lanczos_extremes(al, be)
    assert lo == pytest.approx(0.5, rel=1e-8) and hi == pytest.approx(20.0, rel=1e-8)
    al1, be1 = _textbook_cg_coefficients(A, b, 1)
    lo1, hi1 = api.lanczos_extremes(al1, be1)
    assert lo1 == pytest.approx(b @ A @ b / (b @ b), rel=1e-14) and hi1 == lo1
    # a partial run: Ritz values lie inside the spectrum, the largest close to it
    alp, bep = _textbook_cg_coefficients(A, b, 12)
    lop, hip = api.lanczos_extremes(alp, bep)
    assert 0.5 * (1 - 1e-12) <= lop <= hip <= 20.0 * (1 + 1e-12)


def test_lanczos_extremes_rejects_bad_input():
    lib = N.load()
    d = ctypes.c_double
    a = (d * 2)(1.0, -1.0)
    b = (d * 2)(0.5, 0.5)
    lo, hi = d(0.0), d(0.0)
    assert lib.krr_lanczos_extremes(a, b, 2, ctypes.byref(lo), ctypes.byref(hi)) == N.KRR_EINVAL
    assert lib.krr_lanczos_extremes(a, b, 0, ctypes.byref(lo), ctypes.byref(hi)) == N.KRR_EINVAL
    assert lib.krr_lanczos_extremes(None, b, 1, ctypes.byref(lo), ctypes.byref(hi)) == N.KRR_EINVAL
    assert lib.krr_lanczos_extremes(a, b, 1, ctypes.byref(lo), ctypes.byref(hi)) == N.KRR_OK
    assert lo.value == pytest.approx(1.0) and hi.value == pytest.approx(1.0)
