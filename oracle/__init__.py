"""Double-precision CPU oracle for the regularised Gaussian kernel solver.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
(``paper_1408_1237_amd``) never imports it and shares no code with it; the two
meet only in the seeded input generators of ``paper_1408_1237_amd.workloads``.

The arithmetic lives in ``krr_oracle.c`` (plain FP64 loops, libm ``exp``).  This
module compiles it with gcc on first use and wraps every routine with numpy
argument marshalling; its own arithmetic is limited to library primitives named
where they are used (norms, a symmetric eigenvalue routine).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "krr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")  # AddressSanitizer + UBSan build (host code only)
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile ``krr_oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP); with
    sanitize, into ``liboracle_san.so`` with AddressSanitizer and
    UndefinedBehaviorSanitizer (host C code; load it with the ASan runtime
    preloaded and KRR_ORACLE_SANITIZE=1)."""
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + f".tmp{os.getpid()}"
        opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
        cmd = ["gcc", *opt, "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            sanitize = os.environ.get("KRR_ORACLE_SANITIZE", "0") == "1"
            lib = ctypes.CDLL(build(sanitize=sanitize))
            lib.or_num_threads.restype = _int
            lib.or_set_num_threads.argtypes = [_int]
            lib.or_gauss.restype = _dbl
            lib.or_gauss.argtypes = [_dp, _dp, _int, _dbl]
            lib.or_kernel_matrix.argtypes = [_i64, _i64, _int, _dp, _dp, _dbl, _dp]
            lib.or_mvp.argtypes = [_i64, _i64, _int, _dp, _dp, _dbl, _dbl, _dp, _dp]
            lib.or_mvp_rows.argtypes = [_i64, _int, _dp, _dbl, _dbl, _dp, _i64, _lp, _dp]
            lib.or_cholesky.restype = _int
            lib.or_cholesky.argtypes = [_i64, _dp]
            lib.or_chol_solve.argtypes = [_i64, _dp, _dp, _dp]
            lib.or_cg.restype = _int
            lib.or_cg.argtypes = [_i64, _int, _dp, _dbl, _dbl, _dp, _dp, _int, _dbl, _int,
                                  _ip, _dp, _dp]
            lib.or_fgmres.restype = _int
            lib.or_fgmres.argtypes = [_i64, _int, _dp, _dbl, _dbl, _dp, _dp, _int, _int, _dbl,
                                      _int, _dbl, _int, _dbl, _ip, _dp, _dp, _dp,
                                      _dp, _dp, _dp, _ip]
            lib.or_grad.argtypes = [_i64, _int, _dp, _dbl, _dbl, _dp, _dp, _dp, _dp, _dp]
            lib.or_grad_rows.argtypes = [_i64, _int, _dp, _dbl, _dp, _dp, _i64, _lp, _dp]
            lib.or_fcg.restype = _int
            lib.or_fcg.argtypes = [_i64, _int, _dp, _dbl, _dbl, _dp, _dp, _int, _int, _dbl, _int, _dbl, _int,
                                   _dbl, _ip, _dp, _dp, _dp]
            lib.or_predict.restype = _int
            lib.or_predict.argtypes = [_i64, _i64, _int, _dp, _dp, _dbl, _dbl, _int, _dp, _dp, _dp]
            lib.or_matern.restype = _dbl
            lib.or_matern.argtypes = [_dp, _dp, _int, _dbl]
            lib.or_matern_matrix.argtypes = [_i64, _i64, _int, _dp, _dp, _dbl, _dp]
            lib.or_matern_mvp.argtypes = [_i64, _i64, _int, _dp, _dp, _dbl, _dbl, _dp, _dp]
            lib.or_matern_mvp_rows.argtypes = [_i64, _int, _dp, _dbl, _dbl, _dp, _i64, _lp, _dp]
            _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _pts(x) -> tuple[np.ndarray, int, int]:
    x = _f64(x)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    return x, x.shape[0], x.shape[1]


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(t: int) -> None:
    _load().or_set_num_threads(int(t))


def gauss(a, b, sigma: float) -> float:
    """k(a, b) = exp(-||a-b||^2 / (2 sigma^2)) (eq. Gaussian)."""
    a = _f64(a).ravel()
    b = _f64(b).ravel()
    return _load().or_gauss(_p(a), _p(b), a.size, float(sigma))


def kernel_matrix(xt, sigma: float, xs=None) -> np.ndarray:
    """Explicit K_hat (eq. kernelMatrix); K[i, j] = k(xt_i, xs_j), xs defaults to xt."""
    xt, nt, d = _pts(xt)
    xs, ns, ds = _pts(xt if xs is None else xs)
    assert ds == d
    K = np.empty((nt, ns))
    _load().or_kernel_matrix(nt, ns, d, _p(xt), _p(xs), float(sigma), _p(K))
    return K


def mvp(x, sigma: float, q, shift: float = 0.0, xs=None) -> np.ndarray:
    """On-the-fly y = K_hat q + shift q (square), or K_hat(x, xs) q (rectangular)."""
    xt, nt, d = _pts(x)
    if xs is None:
        xs_, ns = xt, nt
    else:
        xs_, ns, ds = _pts(xs)
        assert ds == d
        if shift != 0.0:
            raise ValueError("shift requires a square product")
    q = _f64(q)
    assert q.shape == (ns,)
    y = np.empty(nt)
    _load().or_mvp(nt, ns, d, _p(xt), _p(xs_), float(sigma), float(shift), _p(q), _p(y))
    return y


def mvp_rows(x, sigma: float, q, rows, shift: float = 0.0) -> np.ndarray:
    """((K_hat + shift I) q)[rows] for a subset of rows."""
    x, n, d = _pts(x)
    q = _f64(q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.size)
    _load().or_mvp_rows(n, d, _p(x), float(sigma), float(shift), _p(q), rows.size,
                        rows.ctypes.data_as(_lp), _p(out))
    return out


def mvp_multi(x, sigma: float, Q, shift: float = 0.0) -> np.ndarray:
    """Y[:, r] = (K_hat + shift I) Q[:, r] for every column of Q."""
    Q = np.asarray(Q, dtype=np.float64)
    return np.stack([mvp(x, sigma, Q[:, r], shift) for r in range(Q.shape[1])], axis=1)


def cholesky(A) -> np.ndarray:
    """Lower Cholesky factor L (A = L L^T), textbook algorithm; raises if A is not PD."""
    L = _f64(A).copy()
    n = L.shape[0]
    rc = _load().or_cholesky(n, _p(L))
    if rc != 0:
        raise np.linalg.LinAlgError(f"not positive definite at pivot {-rc - 1}")
    return L


def chol_solve(L, b) -> np.ndarray:
    L = _f64(L)
    b = _f64(b)
    x = np.empty_like(b)
    _load().or_chol_solve(L.shape[0], _p(L), _p(b), _p(x))
    return x


def direct_solve(x, sigma: float, gamma: float, y) -> np.ndarray:
    """w = (K_hat + gamma I)^{-1} y by explicit K and Cholesky (the paper's "Direct")."""
    K = kernel_matrix(x, sigma)
    K[np.diag_indices_from(K)] += gamma
    return chol_solve(cholesky(K), y)


def cg(x, sigma: float, shift: float, b, maxit: int, tol: float, confirm: bool = True):
    """Textbook CG on (K_hat + shift I) w = b from w = 0.  Returns (w, status, iters, relres, hist)."""
    x, n, d = _pts(x)
    b = _f64(b)
    w = np.empty(n)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    hist = np.full(maxit + 1, np.nan)
    st = _load().or_cg(n, d, _p(x), float(sigma), float(shift), _p(b), _p(w), int(maxit),
                       float(tol), int(bool(confirm)), ctypes.byref(it), ctypes.byref(rel),
                       _p(hist))
    return w, st, it.value, rel.value, hist[: it.value + 1]


def fgmres(x, sigma: float, gamma: float, b, *, m: int = 30, max_outer: int = 300,
           tol: float = 1e-6, inner: str = "cg", delta: float | None = None,
           inner_maxit: int = 10, inner_tol: float | None = None, x0=None,
           want_basis: bool = False) -> dict:
    """Flexible GMRES (Algorithm 1) with an inner CG on K_hat + delta I.

    Defaults follow the paper's rules (section 6): delta = 10 gamma (1e-3 when
    gamma = 0), inner tolerance = 10 x outer tolerance.  ``inner="none"`` gives
    plain GMRES (M = I).
    """
    x, n, d = _pts(x)
    b = _f64(b)
    if delta is None:
        delta = 10.0 * gamma if gamma > 0 else 1e-3
    if inner_tol is None:
        inner_tol = 10.0 * tol
    mode = {"none": 0, "cg": 1}[inner]
    w = np.zeros(n) if x0 is None else _f64(x0).copy()
    info = np.zeros(4, dtype=np.intc)
    est = np.full(max_outer, np.nan)
    tru = np.full(max_outer + 1, np.nan)
    rel = ctypes.c_double(0.0)
    kk = ctypes.c_int(0)
    V = Z = H = None
    if want_basis:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
    st = _load().or_fgmres(
        n, d, _p(x), float(sigma), float(gamma), _p(b), _p(w), int(m), int(max_outer),
        float(tol), mode, float(delta), int(inner_maxit), float(inner_tol),
        info.ctypes.data_as(_ip), _p(est), _p(tru), ctypes.byref(rel),
        _p(V) if want_basis else None, _p(Z) if want_basis else None,
        _p(H) if want_basis else None, ctypes.byref(kk))
    out = dict(w=w, status=int(st), outer=int(info[0]), inner=int(info[1]),
               cycles=int(info[2]), happy=bool(info[3]), relres=rel.value,
               est_hist=est[: info[0]], true_hist=tru[: info[2]])
    if want_basis:
        k = kk.value
        out.update(V=V[: k + 1].T.copy(), Z=Z[:k].T.copy(), H=H[: k + 1, :k].copy(), k=k)
    return out


def fcg(x, sigma: float, gamma: float, b, *, mmax: int = 30, max_outer: int = 300, tol: float = 1e-6,
        inner: str = "cg", delta: float | None = None, inner_maxit: int = 10, inner_tol: float | None = None,
        want_directions: bool = False) -> dict:
    """Flexible CG with re-orthogonalisation over the last mmax directions (see or_fcg)."""
    x, n, d = _pts(x)
    b = _f64(b)
    if delta is None:
        delta = 10.0 * gamma if gamma > 0 else 1e-3
    if inner_tol is None:
        inner_tol = 10.0 * tol
    mode = {"none": 0, "cg": 1}[inner]
    w = np.zeros(n)
    info = np.zeros(2, dtype=np.intc)
    hist = np.full(max_outer + 1, np.nan)
    rel = ctypes.c_double(0.0)
    D = np.zeros((max_outer, n)) if want_directions else None
    st = _load().or_fcg(n, d, _p(x), float(sigma), float(gamma), _p(b), _p(w), int(mmax), int(max_outer),
                        float(tol), mode, float(delta), int(inner_maxit), float(inner_tol),
                        info.ctypes.data_as(_ip), _p(hist), _p(D) if want_directions else None, ctypes.byref(rel))
    out = dict(w=w, status=int(st), outer=int(info[0]), inner=int(info[1]), relres=rel.value,
               hist=hist[: info[0] + 1])
    if want_directions:
        out["D"] = D
    return out


def grad(x, sigma: float, gamma: float, lam, w):
    """(gx (n, d), g_logsigma, g_loggamma) = -lam^T (dK/dtheta) w, explicitly."""
    x, n, d = _pts(x)
    lam = _f64(lam)
    w = _f64(w)
    gx = np.empty((n, d))
    gs = ctypes.c_double(0.0)
    gg = ctypes.c_double(0.0)
    _load().or_grad(n, d, _p(x), float(sigma), float(gamma), _p(lam), _p(w), _p(gx),
                    ctypes.byref(gs), ctypes.byref(gg))
    return gx, gs.value, gg.value


def grad_rows(x, sigma: float, lam, w, rows) -> np.ndarray:
    """The rows `rows` of the point gradient of grad() (shape (len(rows), d))."""
    x, n, d = _pts(x)
    lam = _f64(lam)
    w = _f64(w)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, d))
    _load().or_grad_rows(n, d, _p(x), float(sigma), _p(lam), _p(w), rows.size, rows.ctypes.data_as(_lp), _p(out))
    return out


def true_relres(x, sigma: float, gamma: float, y, w) -> float:
    """||y - (K_hat + gamma I) w|| / ||y|| with the on-the-fly FP64 product."""
    r = _f64(y) - mvp(x, sigma, _f64(w), gamma)
    return float(np.linalg.norm(r) / np.linalg.norm(y))


def eig_extremes(x, sigma: float, gamma: float) -> tuple[float, float]:
    """Smallest and largest eigenvalue of the explicit K_hat + gamma I (eq.
    kernelMatrix); their ratio is the condition number that section 3 ties to
    CG's iteration count.  numpy's symmetric eigenvalue routine is the step."""
    x, n, d = _pts(x)
    ev = np.linalg.eigvalsh(kernel_matrix(x, sigma) + gamma * np.eye(n))
    return float(ev[0]), float(ev[-1])


# ---------------------------------------------------------------- Matern-3/2 (section 6)

def matern(a, b, h: float) -> float:
    """k(a, b) = (1 + sqrt(3) r) exp(-sqrt(3) r), r = ||a - b|| / h (eq. MaternKernel)."""
    a = _f64(a).ravel()
    b = _f64(b).ravel()
    return _load().or_matern(_p(a), _p(b), a.size, float(h))


def matern_matrix(xt, h: float, xs=None) -> np.ndarray:
    """Explicit Matern K_hat; K[i, j] = k(xt_i, xs_j), xs defaults to xt."""
    xt, nt, d = _pts(xt)
    xs, ns, ds = _pts(xt if xs is None else xs)
    assert ds == d
    K = np.empty((nt, ns))
    _load().or_matern_matrix(nt, ns, d, _p(xt), _p(xs), float(h), _p(K))
    return K


def matern_mvp(x, h: float, q, shift: float = 0.0, xs=None) -> np.ndarray:
    """On-the-fly Matern y = K_hat q + shift q (square), or K_hat(x, xs) q."""
    xt, nt, d = _pts(x)
    if xs is None:
        xs_, ns = xt, nt
    else:
        xs_, ns, ds = _pts(xs)
        assert ds == d
        if shift != 0.0:
            raise ValueError("shift requires a square product")
    q = _f64(q)
    assert q.shape == (ns,)
    y = np.empty(nt)
    _load().or_matern_mvp(nt, ns, d, _p(xt), _p(xs_), float(h), float(shift), _p(q), _p(y))
    return y


def matern_mvp_rows(x, h: float, q, rows, shift: float = 0.0) -> np.ndarray:
    """((K_hat + shift I) q)[rows] with the Matern kernel."""
    x, n, d = _pts(x)
    q = _f64(q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.size)
    _load().or_matern_mvp_rows(n, d, _p(x), float(h), float(shift), _p(q), rows.size,
                               rows.ctypes.data_as(_lp), _p(out))
    return out


def matern_direct_solve(x, h: float, gamma: float, y) -> np.ndarray:
    """w = (K_hat + gamma I)^{-1} y with the explicit Matern matrix and Cholesky."""
    K = matern_matrix(x, h)
    K[np.diag_indices_from(K)] += gamma
    return chol_solve(cholesky(K), y)


def predict(x, xs, sigma: float, gamma: float, y, kernel: str = "gauss", want_var: bool = True):
    """GPR posterior mean (eq. GPR_mean) and variance at the test points xs,
    with the explicit matrix and Cholesky (see or_predict)."""
    x, n, d = _pts(x)
    xs, m, ds = _pts(xs)
    assert ds == d
    y = _f64(y)
    mean = np.empty(m)
    var = np.empty(m) if want_var else None
    rc = _load().or_predict(n, m, d, _p(x), _p(xs), float(sigma), float(gamma), {"gauss": 0, "matern32": 1}[kernel],
                            _p(y), _p(mean), _p(var) if want_var else None)
    if rc != 0:
        raise np.linalg.LinAlgError("kernel matrix not positive definite")
    return (mean, var) if want_var else mean
