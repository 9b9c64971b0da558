// Solver drivers on prepared (sorted, zero-padded) point sets.
#pragma once

#include "krylov.h"

namespace krr {

// Status words read back by the host (one copy per outer step).
struct StatusBlock {
    FgmresScalars F;
    CgScalars<float> c32;
    CgScalars<double> c64;
};

// Resolved options (defaults applied).
struct SolverOpts {
    int restart_m = 30;
    int max_outer = 1000;
    double tol = 1e-6;
    int inner = KRR_INNER_CG;
    int inner_prec = KRR_FP32;
    double delta = 0.0;
    int inner_maxit = 10;
    double inner_tol = 1e-5;
    int gs = KRR_GS_MGS;
    int cg_check = 16;
    int kernel = KRR_KERNEL_GAUSS;
};

// Buffers of one solve, carved from the workspace.  b and x are the right-hand
// side and the solution in sorted order.
struct SolverWork {
    double *b = nullptr, *x = nullptr, *w = nullptr;
    double *Ap64 = nullptr, *r64 = nullptr, *p64 = nullptr, *z64 = nullptr;
    double *V = nullptr, *Z = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
    double *hcol = nullptr, *hscr = nullptr;
    float *z32 = nullptr, *r32 = nullptr, *p32 = nullptr, *Ap32 = nullptr;
    uint16_t *p16 = nullptr;
    KmvpScratch ksc;
    StatusBlock *status = nullptr;
    double *cghist = nullptr;  // plain CG: (alpha_k, beta_k) for k < max_outer
    Red R;
};

SolverWork carve_solver(Carver &cv, const Prepared &P, const SolverOpts &o, bool fgmres);

// Map a HIP error to KRR_EHIP inside functions returning a krr_status.
#define KRR_HIP_STATUS(expr)                            \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return KRR_EHIP;          \
    } while (0)

int fgmres_sorted(const Prepared &P, double gamma, bool x0_zero, const SolverOpts &o, const SolverWork &W,
                  krr_info *info, hipStream_t s);
// Flexible CG (the alternative to FGMRES the paper compares, sections 4.2 and
// 5.4): restart_m direction slots, i.e. each new direction is K-orthogonalised
// against up to restart_m - 1 previous ones; x0 = 0; confirmed on the true
// residual (restart from it with an empty window otherwise).  Uses the FGMRES
// workspace.
int fcg_sorted(const Prepared &P, double gamma, const SolverOpts &o, const SolverWork &W, krr_info *info,
               hipStream_t s);
int cg64_sorted(const Prepared &P, double gamma, const SolverOpts &o, const SolverWork &W, krr_info *info,
                hipStream_t s);
// Tune the product plans a solve will use (no-op when already tuned).
hipError_t tune_products(const Prepared &P, const SolverWork &W, bool inner, int inner_prec, hipStream_t s);

// Batched flexible GMRES over many systems and right-hand sides (batched.hip).
size_t batch_workspace_bytes(const krr_points *probs, int nprob, int nrhs, int m);
// FP64 inner products are not batched (KRR_EUNSUPPORTED: the caller solves
// those one at a time).
int batched_fgmres(const krr_points *probs, int nprob, const double *sigma, const double *gamma, int nrhs,
                   const double *const *Y, const int64_t *ldy, double *const *W, const SolverOpts &o,
                   krr_info *infos, void *ws, size_t ws_bytes, hipStream_t s);
// Plain FP64 CG over many systems and right-hand sides at once (the
// comparator of the batched solve).
int batched_cg64(const krr_points *probs, int nprob, const double *sigma, const double *gamma, int nrhs,
                 const double *const *Y, const int64_t *ldy, double *const *W, const SolverOpts &o, krr_info *infos,
                 void *ws, size_t ws_bytes, hipStream_t s);

int cg_inner_sorted(const Prepared &P, int prec, double shift, const double *v_s, double *z_s, int maxit,
                    double tol, const SolverWork &W, krr_info *info, hipStream_t s);

}  // namespace krr
