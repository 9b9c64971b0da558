"""PyTorch-facing wrappers of the C ABI (same names as ``include/krr.h``).

Each function checks tensor placement, shape and dtype, allocates the output
and the workspace as device tensors, and calls the library on the current HIP
stream.  Nothing here computes: there is no CPU path.
"""
from __future__ import annotations

import ctypes

import torch

from . import native as N

_DT = {N.KRR_FP64: torch.float64, N.KRR_FP32: torch.float32, N.KRR_BF16: torch.float32}


def _prec(prec) -> int:
    if isinstance(prec, str):
        return N.PREC[prec]
    return int(prec)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _points(x: torch.Tensor) -> N.Points:
    if not x.is_cuda or x.dtype != torch.float64 or x.dim() != 2 or not x.is_contiguous():
        raise ValueError("points must be a contiguous (n, d) float64 CUDA tensor")
    return N.Points(x.shape[0], x.shape[1], x.data_ptr())


def _vec(v: torch.Tensor, n: int, dtype, name: str) -> torch.Tensor:
    if not v.is_cuda or v.dtype != dtype or v.shape != (n,) or not v.is_contiguous():
        raise ValueError(f"{name} must be a contiguous ({n},) {dtype} CUDA tensor")
    return v


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def make_opts(**kw) -> N.Opts:
    o = N.default_opts()
    for k, v in kw.items():
        if v is None:
            continue
        if k == "inner_prec" and isinstance(v, str):
            v = N.PREC[v]
        if k == "inner" and isinstance(v, str):
            v = {"cg": N.KRR_INNER_CG, "none": N.KRR_INNER_NONE}[v]
        if k == "gs" and isinstance(v, str):
            v = {"mgs": N.KRR_GS_MGS, "cgs2": N.KRR_GS_CGS2}[v]
        if k == "kernel" and isinstance(v, str):
            v = N.KERNEL[v]
        setattr(o, k, v)
    return o


def kmvp_gauss(x: torch.Tensor, sigma: float, q: torch.Tensor, shift: float = 0.0, prec="fp64",
               ws: torch.Tensor | None = None) -> torch.Tensor:
    """y = K_hat q + shift q, computed on the fly on the GPU."""
    return _kmvp_single("kmvp_gauss", x, sigma, q, shift, prec, ws)


def kmvp_matern(x: torch.Tensor, h: float, q: torch.Tensor, shift: float = 0.0, prec="fp64",
                ws: torch.Tensor | None = None) -> torch.Tensor:
    """y = K_hat q + shift q with the Matern-3/2 kernel of length scale h."""
    return _kmvp_single("kmvp_matern", x, h, q, shift, prec, ws)


def _kmvp_single(name, x, sigma, q, shift, prec, ws):
    p = _prec(prec)
    pts = _points(x)
    n = x.shape[0]
    q = _vec(q, n, _DT[p], "q")
    y = torch.empty_like(q)
    need = N.workspace_size(N.KRR_WS_KMVP, [(n, x.shape[1])])
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    N.check(getattr(N.load(), name)(ctypes.byref(pts), float(sigma), float(shift), p, q.data_ptr(), y.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream()), name)
    return y


def kmvp_gauss_multi(x: torch.Tensor, sigma: float, Q: torch.Tensor, shift: float = 0.0, prec="fp64",
                     ws: torch.Tensor | None = None) -> torch.Tensor:
    """Y[:, r] = K_hat Q[:, r] + shift Q[:, r].  Q is (n, nrhs) column-major (Q.t() contiguous)."""
    p = _prec(prec)
    pts = _points(x)
    n, r = Q.shape
    if not Q.is_cuda or Q.dtype != _DT[p] or not Q.t().is_contiguous():
        raise ValueError("Q must be a column-major (n, nrhs) CUDA tensor of the product's dtype")
    Y = torch.empty((r, n), dtype=Q.dtype, device=Q.device).t()
    need = N.workspace_size(N.KRR_WS_KMVP_MULTI, [(n, x.shape[1])], nrhs=r)
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    N.check(N.load().kmvp_gauss_multi(ctypes.byref(pts), float(sigma), float(shift), p, r, Q.data_ptr(), n,
                                      Y.data_ptr(), n, ws.data_ptr(), ws.numel(), _stream()), "kmvp_gauss_multi")
    return Y


def kmvp_gauss_cross(xt: torch.Tensor, xs: torch.Tensor, sigma: float, q: torch.Tensor, prec="fp64",
                     ws: torch.Tensor | None = None) -> torch.Tensor:
    """y = K_hat(targets, sources) q (prediction at new points)."""
    p = _prec(prec)
    pt, ps = _points(xt), _points(xs)
    q = _vec(q, xs.shape[0], _DT[p], "q")
    y = torch.empty(xt.shape[0], dtype=q.dtype, device=q.device)
    need = N.workspace_size(N.KRR_WS_KMVP_CROSS, [(xt.shape[0], xt.shape[1]), (xs.shape[0], xs.shape[1])])
    if ws is None or ws.numel() < need:
        ws = workspace(need, xt.device)
    N.check(N.load().kmvp_gauss_cross(ctypes.byref(pt), ctypes.byref(ps), float(sigma), p, q.data_ptr(),
                                      y.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "kmvp_gauss_cross")
    return y


def kmvp_grad(x: torch.Tensor, sigma: float, gamma: float, lam: torch.Tensor, w: torch.Tensor,
              prec="fp64", ws: torch.Tensor | None = None):
    """(gx (n, d), g_logsigma, g_loggamma) = -lam^T (dK/dtheta) w (device tensors);
    prec "fp64" (default) or "fp32" for the pair loop."""
    p = _prec(prec)
    pts = _points(x)
    n, d = x.shape
    lam = _vec(lam, n, torch.float64, "lam")
    w = _vec(w, n, torch.float64, "w")
    gx = torch.empty((n, d), dtype=torch.float64, device=x.device)
    gs = torch.empty(2, dtype=torch.float64, device=x.device)
    need = N.workspace_size(N.KRR_WS_KMVP_GRAD, [(n, d)])
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    N.check(N.load().kmvp_grad(ctypes.byref(pts), float(sigma), float(gamma), p, lam.data_ptr(), w.data_ptr(),
                               gx.data_ptr(), gs.data_ptr(), gs.data_ptr() + 8, ws.data_ptr(), ws.numel(),
                               _stream()), "kmvp_grad")
    return gx, gs[0], gs[1]


def cg_inner_solve(x: torch.Tensor, sigma: float, shift: float, v: torch.Tensor, maxit: int, tol: float = 0.0,
                   prec="fp32", ws: torch.Tensor | None = None):
    """Truncated CG on (K_hat + shift I) z = v from z = 0.  Returns (z, info dict)."""
    p = _prec(prec)
    pts = _points(x)
    n = x.shape[0]
    v = _vec(v, n, _DT[p], "v")
    z = torch.empty_like(v)
    info = N.Info()
    need = N.workspace_size(N.KRR_WS_CG_INNER, [(n, x.shape[1])])
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    N.check(N.load().cg_inner_solve(ctypes.byref(pts), float(sigma), float(shift), p, v.data_ptr(), z.data_ptr(),
                                    int(maxit), float(tol), ctypes.byref(info), ws.data_ptr(), ws.numel(),
                                    _stream()), "cg_inner_solve")
    return z, info.as_dict()


def fgmres_solve(x: torch.Tensor, sigma: float, gamma: float, b: torch.Tensor, x0: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, **opts):
    """Flexible GMRES (mixed precision) for (K_hat + gamma I) w = b.  Returns (w, info dict)."""
    pts = _points(x)
    n = x.shape[0]
    b = _vec(b, n, torch.float64, "b")
    w = torch.zeros_like(b) if x0 is None else _vec(x0, n, torch.float64, "x0").clone()
    o = make_opts(**opts)
    info = N.Info()
    need = N.workspace_size(N.KRR_WS_FGMRES, [(n, x.shape[1])], opts=o)
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    N.check(N.load().fgmres_solve(ctypes.byref(pts), float(sigma), float(gamma), b.data_ptr(), w.data_ptr(),
                                  ctypes.byref(o), ctypes.byref(info), ws.data_ptr(), ws.numel(), _stream()),
            "fgmres_solve")
    return w, info.as_dict()


def krr_solve(xs, sigmas, gammas, Ys, mode: str = "fgmres", ws: torch.Tensor | None = None,
              return_status: bool = False, **opts):
    """Solve (K_hat_k + gamma_k I) W_k = Y_k for every system k.

    xs: list of (n_k, d_k) float64 CUDA tensors; Ys: list of (n_k,) or (n_k, nrhs)
    column-major float64 tensors (same nrhs for all).  Returns (list of W_k, list of
    info dicts ordered system-major); with return_status also the call's status,
    and a KRR_ENONFINITE status (a non-finite right-hand-side column, the others
    solved) is returned instead of raised.
    """
    modes = {"fgmres": N.KRR_MODE_FGMRES, "cg64": N.KRR_MODE_CG64, "gmres": N.KRR_MODE_GMRES,
             "fcg": N.KRR_MODE_FCG}
    k = len(xs)
    pts = (N.Points * k)(*[_points(x) for x in xs])
    Ys2 = [Y.reshape(-1, 1) if Y.dim() == 1 else Y for Y in Ys]
    Ys2 = [Y if Y.t().is_contiguous() else Y.t().contiguous().t() for Y in Ys2]
    nrhs = Ys2[0].shape[1]
    for x, Y in zip(xs, Ys2):
        if Y.shape != (x.shape[0], nrhs) or Y.dtype != torch.float64 or not Y.is_cuda or not Y.t().is_contiguous():
            raise ValueError("each Y must be a column-major (n_k, nrhs) float64 CUDA tensor")
    Ws = [torch.empty((nrhs, Y.shape[0]), dtype=torch.float64, device=Y.device).t() for Y in Ys2]
    sig = (ctypes.c_double * k)(*[float(s) for s in sigmas])
    gam = (ctypes.c_double * k)(*[float(g) for g in gammas])
    yp = (ctypes.c_void_p * k)(*[Y.data_ptr() for Y in Ys2])
    wp = (ctypes.c_void_p * k)(*[W.data_ptr() for W in Ws])
    ld = (ctypes.c_int64 * k)(*[Y.shape[0] for Y in Ys2])
    o = make_opts(**opts)
    infos = (N.Info * (k * nrhs))()
    need = N.workspace_size(N.KRR_WS_SOLVE, [(x.shape[0], x.shape[1]) for x in xs], nrhs=nrhs, opts=o)
    if ws is None or ws.numel() < need:
        ws = workspace(need, xs[0].device)
    rc = N.load().krr_solve(pts, k, sig, gam, nrhs, yp, ld, wp, modes[mode], ctypes.byref(o), infos,
                            ws.data_ptr(), ws.numel(), _stream())
    if not (return_status and rc == N.KRR_ENONFINITE):
        N.check(rc, "krr_solve")
    Ws = [W.reshape(-1) if Y.dim() == 1 else W for W, Y in zip(Ws, Ys)]
    if return_status:
        return Ws, [i.as_dict() for i in infos], rc
    return Ws, [i.as_dict() for i in infos]


def probe_issue_rates(device="cuda") -> dict:
    """Measured issue rates of the device (see krr_probe_issue_rates): FMA
    lane-ops/s, exp2+FMA pairs/s, matrix-core pairs/s, the FP32 and split-f16
    matrix-core exponent mixes' pairs/s."""
    lib = N.load()
    ws = workspace(int(lib.krr_probe_workspace_size()), torch.device(device))
    rates = (ctypes.c_double * 6)()
    N.check(lib.krr_probe_issue_rates(rates, ws.data_ptr(), ws.numel(), _stream()), "krr_probe_issue_rates")
    return {"fma_lane_ops_s": rates[0], "exp_fma_pairs_s": rates[1], "mfma_pairs_s": rates[2],
            "mg_mix_pairs_s": rates[3], "mh_mix_pairs_s": rates[4], "exp64_fma_pairs_s": rates[5]}


def lanczos_extremes(alpha, beta) -> tuple[float, float]:
    """Extreme eigenvalues of a CG run's Lanczos tridiagonal from its step
    lengths alpha_j and residual ratios beta_j (host computation in the
    library; see krr_lanczos_extremes)."""
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if a.ndim != 1 or b.shape != a.shape:
        raise ValueError("alpha and beta must be 1-D arrays of the same length")
    lo, hi = ctypes.c_double(0.0), ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    N.check(N.load().krr_lanczos_extremes(a.ctypes.data_as(dp), b.ctypes.data_as(dp), int(a.size),
                                          ctypes.byref(lo), ctypes.byref(hi)), "krr_lanczos_extremes")
    return lo.value, hi.value


def krr_predict(x_train: torch.Tensor, x_test: torch.Tensor, sigma: float, gamma: float, w: torch.Tensor,
                want_var: bool = True, ws: torch.Tensor | None = None, **opts):
    """GPR posterior mean K_hat(test, train) w and (want_var) variance at the test
    points.  Returns (mean, var or None, info dicts of the variance solves)."""
    tr, te = _points(x_train), _points(x_test)
    n, m = x_train.shape[0], x_test.shape[0]
    w = _vec(w, n, torch.float64, "w")
    mean = torch.empty(m, dtype=torch.float64, device=x_train.device)
    var = torch.empty(m, dtype=torch.float64, device=x_train.device) if want_var else None
    o = make_opts(**opts)
    need = N.workspace_size(N.KRR_WS_PREDICT, [(n, x_train.shape[1]), (m, x_test.shape[1])], opts=o)
    if ws is None or ws.numel() < need:
        ws = workspace(need, x_train.device)
    infos = (N.Info * m)()
    rc = N.load().krr_predict(ctypes.byref(tr), ctypes.byref(te), float(sigma), float(gamma), w.data_ptr(),
                              mean.data_ptr(), var.data_ptr() if want_var else None, ctypes.byref(o), infos,
                              ws.data_ptr(), ws.numel(), _stream())
    N.check(rc, "krr_predict")
    return mean, var, ([i.as_dict() for i in infos] if want_var else [])
