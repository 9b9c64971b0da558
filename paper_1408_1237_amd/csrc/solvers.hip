// Host drivers of the solvers, on a prepared (sorted, padded) point set:
//  * fgmres_sorted: flexible GMRES (Algorithm 1, section 4.2) with restarts,
//    the inner preconditioner solve of M = K_hat + delta I by truncated CG
//    (sections 4.3, 5.2) in low precision, FP64 outer product, Gram-Schmidt and
//    Givens least squares (section 5.1);
//  * cg_sorted: CG (section 3) in FP64, the unpreconditioned baseline, and the
//    truncated inner CG on its own.
// The drivers only enqueue kernels; they read a small status block back once per
// outer step (FGMRES) or per group of iterations (plain CG).
#include <algorithm>
#include <chrono>
#include <cmath>

#include <cstdio>

#include <vector>
#include "solvers.h"

namespace krr {

static hipError_t read_status(const StatusBlock *dev, StatusBlock &host, hipStream_t s) {
    KRR_HIP(hipMemcpyAsync(&host, dev, sizeof(StatusBlock), hipMemcpyDeviceToHost, s));
    return hipStreamSynchronize(s);
}

SolverWork carve_solver(Carver &cv, const Prepared &P, const SolverOpts &o, bool fgmres) {
    SolverWork W;
    const int64_t np = P.n_pad;
    const int m = o.restart_m;
    W.b = cv.take<double>(np);
    W.x = cv.take<double>(np);
    W.w = cv.take<double>(np);
    W.Ap64 = cv.take<double>(np);
    W.r64 = cv.take<double>(np);
    W.p64 = cv.take<double>(np);
    if (fgmres) {
        W.V = cv.take<double>(static_cast<size_t>(m + 1) * np);
        W.Z = cv.take<double>(static_cast<size_t>(m) * np);
        W.H = cv.take<double>(static_cast<size_t>(m + 1) * m);
        W.cs = cv.take<double>(m);
        W.sn = cv.take<double>(m);
        W.g = cv.take<double>(m + 1);
        W.y = cv.take<double>(m);
        W.hcol = cv.take<double>(m + 2);
        W.hscr = cv.take<double>(m + 2);
        W.z32 = cv.take<float>(np);
        W.r32 = cv.take<float>(np);
        W.p32 = cv.take<float>(np);
        W.Ap32 = cv.take<float>(np);
        W.p16 = cv.take<uint16_t>(np);
        W.z64 = cv.take<double>(np);
    } else {
        W.cghist = cv.take<double>(2 * static_cast<size_t>(o.max_outer > 0 ? o.max_outer : 1));
    }
    W.ksc = carve_kmvp_scratch(cv, P);
    W.status = cv.take<StatusBlock>(1);
    const int nv = (m + 1) > 2 ? (m + 1) : 2;
    W.R.partials = cv.take<double>(Red::partial_count(nv));
    W.R.counters = cv.take<unsigned>(Red::NCOUNTERS);
    return W;
}

hipError_t tune_products(const Prepared &P, const SolverWork &W, bool inner, int inner_prec, hipStream_t s) {
    KRR_HIP(kmvp_tune(P, KRR_FP64, W.b, W.w, W.ksc, s));
    if (inner && inner_prec == KRR_FP64) return hipSuccess;
    if (inner && inner_prec == KRR_FP32) {
        KRR_HIP(zero_bytes(W.p32, P.n_pad * 4, s));
        return kmvp_tune(P, KRR_FP32, W.p32, W.Ap32, W.ksc, s);
    }
    if (inner && inner_prec == KRR_BF16) {
        KRR_HIP(zero_bytes(W.p16, P.n_pad * 2, s));
        return kmvp_tune(P, KRR_BF16, W.p16, W.Ap32, W.ksc, s);
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- inner CG

template <typename T>
static CgVecs<T> inner_vecs(const SolverWork &W, int64_t np, int prec);
template <>
CgVecs<float> inner_vecs<float>(const SolverWork &W, int64_t np, int prec) {
    CgVecs<float> c;
    c.n_pad = np;
    c.x = W.z32;
    c.r = W.r32;
    c.p = W.p32;
    c.Ap = W.Ap32;
    c.p16 = prec == KRR_BF16 ? W.p16 : nullptr;
    c.S = &W.status->c32;
    return c;
}
template <>
CgVecs<double> inner_vecs<double>(const SolverWork &W, int64_t np, int) {
    CgVecs<double> c;
    c.n_pad = np;
    c.x = W.z64;
    c.r = W.r64;
    c.p = W.p64;
    c.Ap = W.Ap64;
    c.S = &W.status->c64;
    return c;
}

// z ~ (K_hat + shift I)^{-1} v, z0 = 0: at most maxit iterations, early stop at
// ||r|| <= tol ||v||.  The result is written (as FP64) to out.
static hipError_t inner_solve(const Prepared &P, int prec, double shift, const double *v, double *out, int maxit,
                              double tol, const SolverWork &W, hipStream_t s) {
    if (prec == KRR_FP64) {
        CgVecs<double> c = inner_vecs<double>(W, P.n_pad, prec);
        KRR_HIP((cg_init<double, double>(c, v, tol, maxit, W.R, s)));
        for (int it = 0; it < maxit; ++it) KRR_HIP(cg_step<double>(P, prec, shift, c, W.ksc, W.R, s));
        return copy_d(P.n_pad, c.x, out, s);
    }
    CgVecs<float> c = inner_vecs<float>(W, P.n_pad, prec);
    KRR_HIP((cg_init<float, double>(c, v, tol, maxit, W.R, s)));
    for (int it = 0; it < maxit; ++it) KRR_HIP(cg_step<float>(P, prec, shift, c, W.ksc, W.R, s));
    return cast_f2d(P.n_pad, c.x, out, s);
}

int cg_inner_sorted(const Prepared &P, int prec, double shift, const double *v_s, double *z_s, int maxit,
                    double tol, const SolverWork &W, krr_info *info, hipStream_t s) {
    KRR_HIP_STATUS(red_init(W.R, s));
    KRR_HIP_STATUS(tune_products(P, W, true, prec, s));
    KRR_HIP_STATUS(inner_solve(P, prec, shift, v_s, z_s, maxit, tol, W, s));
    if (info) {
        StatusBlock st;
        KRR_HIP_STATUS(read_status(W.status, st, s));
        const int iters = prec == KRR_FP64 ? st.c64.iters : st.c32.iters;
        const int stat = prec == KRR_FP64 ? st.c64.status : st.c32.status;
        info->inner_iters = iters;
        info->outer_iters = 0;
        info->status = stat;
        if (prec == KRR_FP64) info->mvp64 = iters;
        else if (prec == KRR_FP32) info->mvp32 = iters;
        else info->mvp16 = iters;
        if (stat != 0) return stat;
    }
    return KRR_OK;
}

// ---------------------------------------------------------------- FGMRES

// Time split of the outer steps: events on the solver's stream around the inner
// solve, the outer product and the orthogonalisation with the Givens update,
// read after the step's status read (the stream is idle then).
struct StepTimer {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    double ms[3] = {0.0, 0.0, 0.0};
    StepTimer() {
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) ok = false;
    }
    ~StepTimer() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    StepTimer(const StepTimer &) = delete;
    StepTimer &operator=(const StepTimer &) = delete;
    void mark(int k, hipStream_t s) {
        if (ok && hipEventRecord(ev[k], s) != hipSuccess) ok = false;
    }
    void collect() {
        if (!ok) return;
        for (int k = 0; k < 3; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) == hipSuccess) ms[k] += t;
        }
    }
};

int fgmres_sorted(const Prepared &P, double gamma, bool x0_zero, const SolverOpts &o, const SolverWork &W,
                  krr_info *info, hipStream_t s) {
    const int64_t np = P.n_pad;
    const int m = o.restart_m;
    FgmresScalars *F = &W.status->F;
    StatusBlock st;
    int64_t mvp64 = 0, mvp_in = 0;
    int outer = 0, inner_total = 0, cycles = 0;
    int result = KRR_NOT_CONVERGED;
    StepTimer tm;

    KRR_HIP_STATUS(red_init(W.R, s));
    KRR_HIP_STATUS(tune_products(P, W, o.inner != KRR_INNER_NONE, o.inner_prec, s));
    // r0 = b - K x0 (section 4.2, first line of the algorithm); r0 lives in W.w
    if (!x0_zero) {
        KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, W.x, W.w, W.ksc, nullptr, s));
        ++mvp64;
    }
    KRR_HIP_STATUS(fg_residual(np, W.b, x0_zero ? nullptr : W.w, W.w, F, W.g, W.R, s));
    KRR_HIP_STATUS(read_status(W.status, st, s));
    if (st.F.nonfinite) return KRR_ENONFINITE;
    double est = st.F.est;
    if (st.F.bnorm == 0.0) {
        KRR_HIP_STATUS(fill_d(W.x, np, 0.0, s));
        est = 0.0;
        result = KRR_OK;
    }
    while (result == KRR_NOT_CONVERGED) {
        if (est <= o.tol) {
            result = KRR_OK;
            break;
        }
        if (outer >= o.max_outer) break;
        KRR_HIP_STATUS(fg_first_basis(np, W.w, W.V, F, s));
        KRR_HIP_STATUS(fill_d(W.g + 1, m, 0.0, s));
        int k = 0;
        bool stop_cycle = false;
        for (int j = 0; j < m && outer < o.max_outer && !stop_cycle; ++j) {
            double *Vj = W.V + static_cast<int64_t>(j) * np;
            double *Zj = W.Z + static_cast<int64_t>(j) * np;
            // inner preconditioner: M_j z_j = v_j
            tm.mark(0, s);
            if (o.inner == KRR_INNER_NONE) {
                KRR_HIP_STATUS(copy_d(np, Vj, Zj, s));
            } else {
                KRR_HIP_STATUS(inner_solve(P, o.inner_prec, o.delta, Vj, Zj, o.inner_maxit, o.inner_tol, W, s));
            }
            tm.mark(1, s);
            // w = K z_j
            KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, Zj, W.w, W.ksc, nullptr, s));
            ++mvp64;
            tm.mark(2, s);
            KRR_HIP_STATUS(fg_orthogonalize(o.gs, np, j, W.w, W.V, W.hcol, W.hscr, F, W.R, s));
            KRR_HIP_STATUS(fg_givens(j, m, W.hcol, W.H, W.cs, W.sn, W.g, F, s));
            KRR_HIP_STATUS(fg_normalize(np, W.w, W.V + static_cast<int64_t>(j + 1) * np, W.hcol, j, F, s));
            tm.mark(3, s);
            KRR_HIP_STATUS(read_status(W.status, st, s));
            tm.collect();
            ++outer;
            k = j + 1;
            if (progress_every() && outer % progress_every() == 0)
                std::fprintf(stderr, "krr fgmres: outer %d cycle %d est %.3e\n", outer, cycles + 1, st.F.est);
            if (o.inner != KRR_INNER_NONE) {
                const int it = o.inner_prec == KRR_FP64 ? st.c64.iters : st.c32.iters;
                inner_total += it;
                mvp_in += it;
            }
            if (st.F.nonfinite) {
                result = KRR_BREAKDOWN;
                k = j;  // drop the column that produced the non-finite value
                stop_cycle = true;
            } else if (st.F.breakdown || st.F.est <= o.tol) {
                stop_cycle = true;
            }
        }
        // y = argmin ||beta e1 - H_bar y||, x = x0 + Z y
        if (k > 0) KRR_HIP_STATUS(fg_update_x(np, k, m, W.H, W.g, W.y, W.Z, W.x, s));
        ++cycles;
        // true residual; also the next cycle's r0
        KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, W.x, W.w, W.ksc, nullptr, s));
        ++mvp64;
        KRR_HIP_STATUS(fg_residual(np, W.b, W.w, W.w, F, W.g, W.R, s));
        KRR_HIP_STATUS(read_status(W.status, st, s));
        est = st.F.est;
        if (st.F.nonfinite) result = KRR_BREAKDOWN;
        if (result == KRR_BREAKDOWN) break;
    }
    if (info) {
        info->status = result;
        info->outer_iters = outer;
        info->inner_iters = inner_total;
        info->cycles = cycles;
        info->mvp64 = mvp64;
        info->mvp32 = (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_FP32) ? mvp_in : 0;
        info->mvp16 = (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_BF16) ? mvp_in : 0;
        if (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_FP64) info->mvp64 += mvp_in;
        info->relres_true = est;
        info->relres_est = est;
        info->t_inner_ms = tm.ms[0];
        info->t_outer_ms = tm.ms[1];
        info->t_ortho_ms = tm.ms[2];
    }
    return result;
}

// ---------------------------------------------------------------- flexible CG

int fcg_sorted(const Prepared &P, double gamma, const SolverOpts &o, const SolverWork &W, krr_info *info,
               hipStream_t s) {
    const int64_t np = P.n_pad;
    const int m = o.restart_m;
    FgmresScalars *F = &W.status->F;
    double *r = W.V + static_cast<int64_t>(m) * np;  // slots 0..m-1 of V hold the directions d_k
    double *z = W.w;
    double *dq = W.H, *alpha = W.H + m;
    StatusBlock st;
    int64_t mvp64 = 0, mvp_in = 0;
    int it = 0, since = 0, inner_total = 0, restarts = 0;
    int result = KRR_NOT_CONVERGED;

    KRR_HIP_STATUS(red_init(W.R, s));
    KRR_HIP_STATUS(tune_products(P, W, o.inner != KRR_INNER_NONE, o.inner_prec, s));
    KRR_HIP_STATUS(fill_d(W.x, np, 0.0, s));
    KRR_HIP_STATUS(fg_residual(np, W.b, nullptr, r, F, W.g, W.R, s));
    KRR_HIP_STATUS(read_status(W.status, st, s));
    if (st.F.nonfinite) return KRR_ENONFINITE;
    double est = st.F.bnorm == 0.0 ? 0.0 : st.F.est;
    for (;;) {
        if (est <= o.tol) {
            if (st.F.bnorm == 0.0) {
                result = KRR_OK;
                break;
            }
            // confirm with the true residual b - K x; restart from it otherwise
            KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, W.x, W.Ap64, W.ksc, nullptr, s));
            ++mvp64;
            KRR_HIP_STATUS(fg_residual(np, W.b, W.Ap64, r, F, W.g, W.R, s));
            KRR_HIP_STATUS(read_status(W.status, st, s));
            est = st.F.est;
            if (est <= o.tol) {
                result = KRR_OK;
                break;
            }
            since = 0;
            ++restarts;
        }
        if (it >= o.max_outer) break;
        // z = M^-1 r (inner CG on K_hat + delta I), or z = r
        if (o.inner == KRR_INNER_NONE) {
            KRR_HIP_STATUS(copy_d(np, r, z, s));
        } else {
            KRR_HIP_STATUS(inner_solve(P, o.inner_prec, o.delta, r, z, o.inner_maxit, o.inner_tol, W, s));
        }
        const int cur = since % m;
        const int nslots = since < m ? since : m;
        KRR_HIP_STATUS(fcg_direction(np, nslots, cur, z, W.V, W.Z, W.hcol, W.y, W.hscr, dq, W.R, s));
        double *dcur = W.V + static_cast<int64_t>(cur) * np;
        double *qcur = W.Z + static_cast<int64_t>(cur) * np;
        KRR_HIP_STATUS(copy_d(np, z, dcur, s));
        KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, dcur, qcur, W.ksc, nullptr, s));
        ++mvp64;
        KRR_HIP_STATUS(fcg_step(np, dcur, qcur, W.x, r, dq, cur, alpha, F, W.R, s));
        KRR_HIP_STATUS(read_status(W.status, st, s));
        ++it;
        ++since;
        if (o.inner != KRR_INNER_NONE) {
            const int k = o.inner_prec == KRR_FP64 ? st.c64.iters : st.c32.iters;
            inner_total += k;
            mvp_in += k;
        }
        if (st.F.breakdown || st.F.nonfinite) {
            result = KRR_BREAKDOWN;
            break;
        }
        est = st.F.est;
        if (progress_every() && it % progress_every() == 0)
            std::fprintf(stderr, "krr fcg: iteration %d rel. residual (recursive) %.3e\n", it, est);
    }
    if (result == KRR_NOT_CONVERGED) {  // report the true residual of the last iterate
        KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, W.x, W.Ap64, W.ksc, nullptr, s));
        ++mvp64;
        KRR_HIP_STATUS(fg_residual(np, W.b, W.Ap64, r, F, W.g, W.R, s));
        KRR_HIP_STATUS(read_status(W.status, st, s));
        est = st.F.est;
    }
    if (info) {
        info->status = result;
        info->outer_iters = it;
        info->inner_iters = inner_total;
        info->cycles = restarts + 1;
        info->mvp64 = mvp64;
        info->mvp32 = (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_FP32) ? mvp_in : 0;
        info->mvp16 = (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_BF16) ? mvp_in : 0;
        if (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_FP64) info->mvp64 += mvp_in;
        info->relres_true = est;
        info->relres_est = est;
    }
    return result;
}

// ---------------------------------------------------------------- plain FP64 CG

int cg64_sorted(const Prepared &P, double gamma, const SolverOpts &o, const SolverWork &W, krr_info *info,
                hipStream_t s) {
    const int64_t np = P.n_pad;
    CgVecs<double> c;
    c.n_pad = np;
    c.x = W.x;
    c.r = W.r64;
    c.p = W.p64;
    c.Ap = W.Ap64;
    c.S = &W.status->c64;
    c.hist = W.cghist;
    c.hist_cap = o.max_outer;
    StatusBlock st;
    int64_t mvp64 = 0;
    int lanczos_k = -1;  // iterations of the first CG run (before any restart)
    int cycles = 1;
    int result = KRR_NOT_CONVERGED;
    double relres = 1.0;
    const int check = o.cg_check > 0 ? o.cg_check : 16;

    KRR_HIP_STATUS(red_init(W.R, s));
    KRR_HIP_STATUS(tune_products(P, W, false, KRR_FP64, s));
    KRR_HIP_STATUS((cg_init<double, double>(c, W.b, o.tol, o.max_outer, W.R, s)));
    KRR_HIP_STATUS(read_status(W.status, st, s));
    if (st.c64.status == KRR_ENONFINITE) return KRR_ENONFINITE;
    if (st.c64.rr0 == 0.0) {
        result = KRR_OK;
        relres = 0.0;
    }
    int last_iters = 0;
    while (result == KRR_NOT_CONVERGED) {
        for (int k = 0; k < check; ++k) KRR_HIP_STATUS(cg_step<double>(P, KRR_FP64, gamma, c, W.ksc, W.R, s));
        KRR_HIP_STATUS(read_status(W.status, st, s));
        mvp64 += st.c64.iters - last_iters;
        if (progress_every() && st.c64.iters / progress_every() != last_iters / progress_every())
            std::fprintf(stderr, "krr cg64: iteration %d rel. residual (recursive) %.3e\n", st.c64.iters,
                         std::sqrt(st.c64.rr / st.c64.rr0));
        last_iters = st.c64.iters;
        if (st.c64.status == KRR_BREAKDOWN) {
            result = KRR_BREAKDOWN;
            break;
        }
        if (st.c64.candidate || st.c64.active == 0) {
            // confirm with the true residual b - K x; restart from it if needed
            if (lanczos_k < 0) lanczos_k = st.c64.iters;
            KRR_HIP_STATUS(kmvp_sorted(P, KRR_FP64, gamma, c.x, W.Ap64, W.ksc, nullptr, s));
            ++mvp64;
            KRR_HIP_STATUS(cg_restart<double>(c, W.b, W.Ap64, W.R, s));
            KRR_HIP_STATUS(read_status(W.status, st, s));
            relres = std::sqrt(st.c64.rr / st.c64.rr0);
            if (st.c64.candidate) {
                result = KRR_OK;
                break;
            }
            if (st.c64.iters >= o.max_outer) break;
            ++cycles;
        }
    }
    if (info) {
        info->status = result;
        info->outer_iters = st.c64.iters;
        info->inner_iters = 0;
        info->cycles = cycles;
        info->mvp64 = mvp64;
        info->mvp32 = info->mvp16 = 0;
        info->relres_true = relres;
        info->relres_est = std::sqrt(st.c64.rr / st.c64.rr0);
        info->lambda_min_est = info->lambda_max_est = 0.0;
        const int k = std::min(lanczos_k < 0 ? st.c64.iters : lanczos_k, o.max_outer);
        if (k > 0) {
            std::vector<double> h(2 * static_cast<size_t>(k));
            KRR_HIP_STATUS(hipMemcpyAsync(h.data(), W.cghist, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            KRR_HIP_STATUS(hipStreamSynchronize(s));
            std::vector<double> a(k), b(k);
            for (int j = 0; j < k; ++j) {
                a[j] = h[2 * j];
                b[j] = h[2 * j + 1];
            }
            double lo = 0.0, hi = 0.0;
            if (krr_lanczos_extremes(a.data(), b.data(), k, &lo, &hi) == KRR_OK) {
                info->lambda_min_est = lo;
                info->lambda_max_est = hi;
            }
        }
    }
    return result;
}

}  // namespace krr
