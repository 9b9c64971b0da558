// Launchers of the Krylov vector kernels (krylov.hip) and the solver drivers
// (solvers.hip).
#pragma once

#include "krr_internal.h"

namespace krr {

// Reduction scratch of one solver: partial sums (VEC_BLOCKS * 4 doubles) and
// the last-block counters (zeroed by red_init, reset by every reduction).
struct Red {
    static constexpr int NCOUNTERS = 16;
    double *partials = nullptr;
    unsigned *counters = nullptr;
    static size_t partial_count(int nv_max) { return static_cast<size_t>(VEC_BLOCKS) * nv_max; }
};

// Vectors of one CG solve (T = float: inner solve; double: plain solver).
template <typename T>
struct CgVecs {
    int64_t n_pad = 0;
    T *x = nullptr, *r = nullptr, *p = nullptr, *Ap = nullptr;
    uint16_t *p16 = nullptr;  // only for the bf16 product
    CgScalars<T> *S = nullptr;
    double *hist = nullptr;   // optional (alpha_k, beta_k) history, hist_cap pairs
    int hist_cap = 0;
};

int vec_blocks(int64_t n_pad);
hipError_t red_init(const Red &R, hipStream_t s);

template <typename T, typename TV>
hipError_t cg_init(const CgVecs<T> &c, const TV *rhs, double tol, int maxit, const Red &R, hipStream_t s);
template <typename T>
hipError_t cg_step(const Prepared &P, int prec, double shift, const CgVecs<T> &c, const KmvpScratch &sc,
                   const Red &R, hipStream_t s);
template <typename T>
hipError_t cg_restart(const CgVecs<T> &c, const T *b, const T *Kx, const Red &R, hipStream_t s);

hipError_t fg_residual(int64_t n_pad, const double *b, const double *Kx, double *r, FgmresScalars *F, double *g,
                       const Red &R, hipStream_t s);
hipError_t fg_first_basis(int64_t n_pad, const double *r, double *v, const FgmresScalars *F, hipStream_t s);
hipError_t cast_f2d(int64_t n_pad, const float *z, double *Zj, hipStream_t s);
hipError_t copy_d(int64_t n_pad, const double *a, double *b, hipStream_t s);
hipError_t fill_d(double *p, int64_t n, double v, hipStream_t s);
hipError_t zero_bytes(void *p, int64_t n, hipStream_t s);  // fill kernel (no memset nodes)
hipError_t fg_orthogonalize(int gs, int64_t n_pad, int j, double *w, const double *V, double *hcol, double *hscratch,
                            FgmresScalars *F, const Red &R, hipStream_t s);
hipError_t fg_givens(int j, int m, const double *hcol, double *H, double *cs, double *sn, double *g,
                     FgmresScalars *F, hipStream_t s);
hipError_t fg_normalize(int64_t n_pad, const double *w, double *vnext, const double *hcol, int j,
                        const FgmresScalars *F, hipStream_t s);
hipError_t fg_update_x(int64_t n_pad, int k, int m, const double *H, const double *g, double *y, const double *Z,
                       double *x, hipStream_t s);
// Flexible CG: z -= D beta over nslots stored directions (beta_k = z.q_k / d_k.q_k,
// 0 for slot cur); then alpha = d.r / d.q (dq[cur] kept), x += alpha d, r -= alpha q,
// F->est = ||r|| / ||b||, F->breakdown on d.q <= 0.
hipError_t fcg_direction(int64_t n_pad, int nslots, int cur, double *z, const double *D, const double *Q,
                         double *hcol, double *hpass, double *dq_beta_scratch, const double *dq, const Red &R,
                         hipStream_t s);
hipError_t fcg_step(int64_t n_pad, const double *d, const double *q, double *x, double *r, double *dq, int cur,
                    double *alpha, FgmresScalars *F, const Red &R, hipStream_t s);

}  // namespace krr
