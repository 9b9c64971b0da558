// Batched flexible GMRES: many independent systems (K_hat_k + gamma_k I) W_k = Y_k
// with several right-hand sides each, advanced together (the paper solves one
// kriging system per week, section 6.3; the variance of eq. GPR_mean needs one
// solve per test point, section 2.1).
//
// Layout: every (system k, column r) pair is a segment of length n_pad_k in one
// concatenated vector; the columns of a system are consecutive (a column-major
// n_pad_k x Rp block, Rp = 16 ceil(nrhs / 16)), so the kernel products of a
// system are one multi-RHS matrix-core launch.  Reductions are segmented: every
// 256-element chunk belongs to one column; a block reduces its chunk and the
// last block of the column (per-column counter) adds the column's partials in
// order.  All solver scalars are per column in device memory; a column that has
// converged (or broken down) drops out through its active flags.  The inner CG
// sequence (its products and vector kernels on fixed buffers) is captured once
// in a HIP graph and replayed at every outer step.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "kmvp_multi.h"
#include "solvers.h"

namespace krr {

namespace {

struct BCols {  // per-column device state (arrays of C entries unless noted)
    // inner CG (FP32)
    float *rr, *rr0, *thresh, *alpha, *beta;
    int *cg_active, *cg_iters;
    // FGMRES
    double *bnorm, *beta_o, *est, *wnorm0;
    int *breakdown, *in_cycle, *kcol, *valid;
    int *status;                      // KRR_BREAKDOWN / KRR_ENONFINITE once a column is retired, else 0
    int *col_outer, *col_inner, *col_mvp64, *col_cycles;  // per-column counts
    double *H, *cs, *sn, *g, *y, *hcol;  // C x (m+1) x m, C x m, C x m, C x (m+1), C x m, C x (m+2)
    double *gcoef;                    // C x (m+2): coefficients of the current Gram-Schmidt pass
    // plain FP64 CG
    double *rr64, *alpha64, *beta64;
    int *cand, *restart;              // needs a true-residual check; direction restarts from r
    int *chunk_col;    // [nchunks]
    int *col_chunk0;   // [C]
    int *col_nchunk;   // [C]
    int64_t *col_off;  // [C] element offset of the column
    double *partials;  // [nchunks * pstride]
    int pstride;       // partial sums per chunk (m + 2: Gram-Schmidt block dots)
    int *summary;      // [4]: columns in their cycle, non-finite columns, active CG columns, CG columns to check
};

__device__ __forceinline__ double bwave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o /= 2) v += __shfl_xor(v, o, WAVE);
    return v;
}

template <int NV>
__device__ __forceinline__ void bblock_sum(double (&v)[NV]) {
    __shared__ double sh[NV][BLOCK / WAVE];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = bwave_sum(v[k]);
    __syncthreads();
    if (threadIdx.x % WAVE == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][threadIdx.x / WAVE] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < BLOCK / WAVE; ++w) s += sh[k][w];
            v[k] = s;
        }
}

// Segmented sums in two kernels, with no fences or atomics: a chunk kernel
// (one block per 256-element chunk, every chunk inside one column) writes its
// block sums to partials[chunk]; the column kernel that follows (one wave per
// column) adds the column's chunk sums in a fixed order and runs the epilogue.
template <int NV>
__device__ __forceinline__ void seg_partial(double (&v)[NV], const BCols &B) {
    bblock_sum(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) B.partials[static_cast<int64_t>(blockIdx.x) * B.pstride + k] = v[k];
}

// Column of this wave (-1 past the last column).
__device__ __forceinline__ int wave_col(int C) {
    const int c = blockIdx.x * (BLOCK / WAVE) + static_cast<int>(threadIdx.x) / WAVE;
    return c < C ? c : -1;
}

// Sum k of the column's chunks, in every lane (lane l adds chunks l, l + 64,
// ...; then a fixed butterfly).  Called by all lanes of the wave.
__device__ __forceinline__ double col_sum(const BCols &B, int c, int k) {
    const int c0 = B.col_chunk0[c], nc = B.col_nchunk[c];
    const int lane = static_cast<int>(threadIdx.x) % WAVE;
    double s = 0.0;
    for (int q = lane; q < nc; q += WAVE) s += B.partials[static_cast<int64_t>(c0 + q) * B.pstride + k];
    return bwave_sum(s);
}

template <int NV>
__device__ __forceinline__ void col_total(const BCols &B, int c, double (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = col_sum(B, c, k);
}

#define BCHUNK                                                        \
    const int c = B.chunk_col[blockIdx.x];                            \
    const int64_t e = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x

// ---------------------------------------------------------------- inner CG (FP32)

__global__ __launch_bounds__(BLOCK) void kb_cg_init(BCols B, const double *__restrict__ vin, float *z, float *r,
                                                    float *p) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const float v = static_cast<float>(vin[e]);
    z[e] = 0.f;
    r[e] = v;
    p[e] = v;
    double acc[1] = {static_cast<double>(v) * v};
    seg_partial(acc, B);
}

__global__ __launch_bounds__(BLOCK) void kb_cg_init_col(BCols B, int C, double tol2, int maxit) {
    const int c = wave_col(C);
    if (c < 0 || !B.in_cycle[c]) return;
    double acc[1];
    col_total(B, c, acc);
    if (threadIdx.x % WAVE == 0) {
        const float rr = static_cast<float>(acc[0]);
        B.rr[c] = rr;
        B.rr0[c] = rr;
        B.thresh[c] = static_cast<float>(tol2 * acc[0]);
        B.cg_iters[c] = 0;
        B.cg_active[c] = (rr > 0.f && maxit > 0) ? 1 : 0;
    }
}

__global__ __launch_bounds__(BLOCK) void kb_cg_alpha(BCols B, const float *__restrict__ p,
                                                     const float *__restrict__ Ap) {
    BCHUNK;
    if (!B.in_cycle[c] || !B.cg_active[c]) return;
    double acc[1] = {static_cast<double>(p[e]) * Ap[e]};
    seg_partial(acc, B);
}

__global__ __launch_bounds__(BLOCK) void kb_cg_alpha_col(BCols B, int C) {
    const int c = wave_col(C);
    if (c < 0 || !B.in_cycle[c] || !B.cg_active[c]) return;
    double acc[1];
    col_total(B, c, acc);
    if (threadIdx.x % WAVE == 0) {
        const float pAp = static_cast<float>(acc[0]);
        if (!(pAp > 0.f) || !isfinite(pAp))
            B.cg_active[c] = 0;
        else
            B.alpha[c] = B.rr[c] / pAp;
    }
}

__global__ __launch_bounds__(BLOCK) void kb_cg_update(BCols B, float *z, float *r, const float *__restrict__ p,
                                                      const float *__restrict__ Ap) {
    BCHUNK;
    if (!B.in_cycle[c] || !B.cg_active[c]) return;
    const float a = B.alpha[c];
    z[e] += a * p[e];
    const float ri = r[e] - a * Ap[e];
    r[e] = ri;
    double acc[1] = {static_cast<double>(ri) * ri};
    seg_partial(acc, B);
}

// Also retires a column whose CG reached maxit (keeps the products of the next
// iteration off it).
__global__ __launch_bounds__(BLOCK) void kb_cg_update_col(BCols B, int C, int maxit) {
    const int c = wave_col(C);
    if (c < 0 || !B.in_cycle[c] || !B.cg_active[c]) return;
    double acc[1];
    col_total(B, c, acc);
    if (threadIdx.x % WAVE == 0) {
        const float rr = static_cast<float>(acc[0]);
        B.beta[c] = rr / B.rr[c];
        B.rr[c] = rr;
        const int it = B.cg_iters[c] + 1;
        B.cg_iters[c] = it;
        if (!isfinite(rr) || rr <= B.thresh[c] || it >= maxit) B.cg_active[c] = 0;
    }
}

__global__ __launch_bounds__(BLOCK) void kb_cg_pupdate(BCols B, const float *__restrict__ r, float *p) {
    BCHUNK;
    if (!B.in_cycle[c] || !B.cg_active[c]) return;
    p[e] = r[e] + B.beta[c] * p[e];
}

// ---------------------------------------------------------------- FGMRES (FP64)

// r = b - Kx (Kx may be null), per column beta, bnorm, est; starts the cycle of
// every valid column that is above the tolerance.  At a cycle end (Kx given)
// a column that took no step keeps its state: its x, and so its residual, did
// not change (its product was skipped).
__global__ __launch_bounds__(BLOCK) void kb_residual(BCols B, const double *__restrict__ b, const double *Kx,
                                                     double *r) {
    BCHUNK;
    if (!B.valid[c]) {
        r[e] = 0.0;
        return;
    }
    if (Kx != nullptr && B.kcol[c] == 0) return;
    const double bi = b[e];
    const double v = Kx ? bi - Kx[e] : bi;
    r[e] = v;
    double acc[2] = {v * v, bi * bi};
    seg_partial(acc, B);
}

// Column epilogue of kb_residual.  A column whose right-hand side is not finite
// (at the start) is retired with KRR_ENONFINITE and never touched again; one
// whose residual turns non-finite later, or that broke down in its Givens step,
// is retired with KRR_BREAKDOWN and keeps its last finite iterate.
__global__ __launch_bounds__(BLOCK) void kb_residual_col(BCols B, int C, int cycle_end, int m, double tol) {
    const int c = wave_col(C);
    if (c < 0 || !B.valid[c] || (cycle_end && B.kcol[c] == 0)) return;
    double acc[2];
    col_total(B, c, acc);
    if (threadIdx.x % WAVE == 0) {
        const double beta = sqrt(acc[0]), bn = sqrt(acc[1]);
        const double est = !isfinite(beta) || !isfinite(bn) ? NAN : (bn > 0.0 ? beta / bn : 0.0);
        B.kcol[c] = 0;
        B.breakdown[c] = 0;
        B.in_cycle[c] = 0;
        if (cycle_end) {
            B.col_mvp64[c] += 1;
            B.col_cycles[c] += 1;
        }
        if (!isfinite(est)) {
            B.status[c] = cycle_end ? KRR_BREAKDOWN : KRR_ENONFINITE;
            if (!cycle_end) B.valid[c] = 0;
            return;
        }
        B.beta_o[c] = beta;
        B.bnorm[c] = bn;
        B.est[c] = est;
        if (B.status[c] != 0) return;
        B.in_cycle[c] = est > tol ? 1 : 0;
        double *g = B.g + static_cast<int64_t>(c) * (m + 1);
        g[0] = beta;
        for (int k = 1; k <= m; ++k) g[k] = 0.0;
    }
}

__global__ __launch_bounds__(BLOCK) void kb_first_basis(BCols B, const double *__restrict__ r, double *v0) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    v0[e] = r[e] / B.beta_o[c];
}

// z (FP32 inner solution) -> Z_j; the column's first chunk block also adds the
// inner iterations of this step to its count.
__global__ __launch_bounds__(BLOCK) void kb_cast_z(BCols B, const float *__restrict__ z, double *Zj) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    Zj[e] = static_cast<double>(z[e]);
    if (threadIdx.x == 0 && static_cast<int>(blockIdx.x) == B.col_chunk0[c]) B.col_inner[c] += B.cg_iters[c];
}

__global__ __launch_bounds__(BLOCK) void kb_copy(BCols B, const double *__restrict__ a, double *bout) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    bout[e] = a[e];
}

// Modified Gram-Schmidt, one pass per basis vector: h_0 = w.v_0 (and ||w||),
// then for i = 0..j-1: w -= h_i v_i, h_{i+1} = w.v_{i+1}; last: w -= h_j v_j,
// h_{j+1} = ||w||.  site: 0 first, 1 step, 2 last.
__global__ __launch_bounds__(BLOCK) void kb_mgs_first(BCols B, const double *__restrict__ w,
                                                      const double *__restrict__ v0) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const double wi = w[e];
    double acc[2] = {wi * v0[e], wi * wi};
    seg_partial(acc, B);
}

__global__ __launch_bounds__(BLOCK) void kb_mgs_step(BCols B, double *w, const double *__restrict__ vi,
                                                     const double *__restrict__ vnext, int i_, int m) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const double *hc = B.hcol + static_cast<int64_t>(c) * (m + 2);
    const double wi = w[e] - hc[i_] * vi[e];
    w[e] = wi;
    double acc[1] = {wi * vnext[e]};
    seg_partial(acc, B);
}

__global__ __launch_bounds__(BLOCK) void kb_mgs_last(BCols B, double *w, const double *__restrict__ vj, int j,
                                                     int m) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const double *hc = B.hcol + static_cast<int64_t>(c) * (m + 2);
    const double wi = w[e] - hc[j] * vj[e];
    w[e] = wi;
    double acc[1] = {wi * wi};
    seg_partial(acc, B);
}

// Column epilogue of the three Gram-Schmidt passes: writes hcol[idx] (site 0:
// also ||w|| before orthogonalisation; site 2: the norm).
__global__ __launch_bounds__(BLOCK) void kb_mgs_col(BCols B, int C, int site, int idx, int m) {
    const int c = wave_col(C);
    if (c < 0 || !B.in_cycle[c]) return;
    double acc[2];
    if (site == 0) {
        col_total(B, c, acc);
    } else {
        double one[1];
        col_total(B, c, one);
        acc[0] = one[0];
    }
    if (threadIdx.x % WAVE == 0) {
        double *hc = B.hcol + static_cast<int64_t>(c) * (m + 2);
        if (site == 0) {
            hc[0] = acc[0];
            B.wnorm0[c] = sqrt(acc[1]);
        } else if (site == 1) {
            hc[idx] = acc[0];
        } else {
            hc[idx] = sqrt(acc[0]);
        }
    }
}

// Classical Gram-Schmidt applied twice (the blocked alternative to MGS): per
// pass, the dot products of w with v_0..v_j in one sweep (and, in the first
// pass, w.w for the breakdown test), then w -= sum_i g_i v_i.  Chunk kernel:
// block sums of w v_i (i <= j) and of w w (slot j + 1, when wsq).
__global__ __launch_bounds__(BLOCK) void kb_gs_dot(BCols B, const double *__restrict__ w,
                                                   const double *__restrict__ V, int64_t LL, int j, int wsq) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const double wi = w[e];
    const int nv = j + 1 + wsq;
    double *out = B.partials + static_cast<int64_t>(blockIdx.x) * B.pstride;
    for (int i0 = 0; i0 < nv; i0 += 8) {
        double acc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = i0 + k;
            acc[k] = i <= j ? wi * V[static_cast<int64_t>(i) * LL + e] : (i < nv ? wi * wi : 0.0);
        }
        bblock_sum(acc);
        if (threadIdx.x == 0)
            for (int k = 0; k < 8 && i0 + k < nv; ++k) out[i0 + k] = acc[k];
    }
}

// Column epilogue of a pass: g_i for i <= j into gcoef; pass 0 stores them in
// hcol (and ||w|| before orthogonalisation), pass 1 adds them.
__global__ __launch_bounds__(BLOCK) void kb_gs_col(BCols B, int C, int j, int pass, int m) {
    const int c = wave_col(C);
    if (c < 0 || !B.in_cycle[c]) return;
    double *hc = B.hcol + static_cast<int64_t>(c) * (m + 2);
    double *gc = B.gcoef + static_cast<int64_t>(c) * (m + 2);
    const int nv = j + 1 + (pass == 0 ? 1 : 0);
    for (int i = 0; i < nv; ++i) {
        const double s = col_sum(B, c, i);
        if (threadIdx.x % WAVE == 0) {
            if (i <= j) {
                gc[i] = s;
                hc[i] = pass == 0 ? s : hc[i] + s;
            } else {
                B.wnorm0[c] = sqrt(s);
            }
        }
    }
}

__global__ __launch_bounds__(BLOCK) void kb_gs_update(BCols B, double *w, const double *__restrict__ V, int64_t LL,
                                                      int j, int m) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const double *gc = B.gcoef + static_cast<int64_t>(c) * (m + 2);
    double v = w[e];
    for (int i = 0; i <= j; ++i) v -= gc[i] * V[static_cast<int64_t>(i) * LL + e];
    w[e] = v;
}

__global__ __launch_bounds__(BLOCK) void kb_wsq(BCols B, const double *__restrict__ w) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    const double wi = w[e];
    double acc[1] = {wi * wi};
    seg_partial(acc, B);
}

// Givens step of every column in its cycle (one thread per column); a column
// leaves the cycle on convergence of its estimate or on breakdown, and is
// retired (KRR_BREAKDOWN, its steps before this one kept) on a non-finite value.
__global__ void kb_givens(BCols B, int C, int j, int m, double tol) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C || !B.in_cycle[c]) return;
    const double *hc = B.hcol + static_cast<int64_t>(c) * (m + 2);
    double *col = B.H + (static_cast<int64_t>(c) * m + j) * (m + 1);
    double *cs = B.cs + static_cast<int64_t>(c) * m, *sn = B.sn + static_cast<int64_t>(c) * m;
    double *g = B.g + static_cast<int64_t>(c) * (m + 1);
    B.col_outer[c] += 1;
    B.col_mvp64[c] += 1;
    for (int i = 0; i <= j + 1; ++i) col[i] = hc[i];
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double rho = sqrt(a * a + b * b);
    const double cj = a / rho, sj = b / rho;
    const double est = fabs(-sj * g[j]) / B.bnorm[c];
    if (!isfinite(est) || !isfinite(rho)) {
        B.status[c] = KRR_BREAKDOWN;
        B.kcol[c] = j;
        B.in_cycle[c] = 0;
        return;
    }
    cs[j] = cj;
    sn[j] = sj;
    col[j] = rho;
    col[j + 1] = 0.0;
    g[j + 1] = -sj * g[j];
    g[j] = cj * g[j];
    B.est[c] = est;
    B.kcol[c] = j + 1;
    const int brk = (hc[j + 1] > 1e-14 * B.wnorm0[c]) ? 0 : 1;
    B.breakdown[c] = brk;
    if (brk || est <= tol) B.in_cycle[c] = 0;
}

__global__ __launch_bounds__(BLOCK) void kb_normalize(BCols B, const double *__restrict__ w, double *vnext, int j,
                                                      int m) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    vnext[e] = w[e] / B.hcol[static_cast<int64_t>(c) * (m + 2) + j + 1];
}

// y_c = R^{-1} g over the column's own k steps (one thread per column).
__global__ void kb_backsolve(BCols B, int C, int m) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C || !B.valid[c]) return;
    const int k = B.kcol[c];
    const double *H = B.H + static_cast<int64_t>(c) * m * (m + 1);
    const double *g = B.g + static_cast<int64_t>(c) * (m + 1);
    double *y = B.y + static_cast<int64_t>(c) * m;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int t = i + 1; t < k; ++t) s -= H[static_cast<int64_t>(t) * (m + 1) + i] * y[t];
        y[i] = s / H[static_cast<int64_t>(i) * (m + 1) + i];
    }
}

__global__ __launch_bounds__(BLOCK) void kb_update_x(BCols B, const double *__restrict__ Z, int64_t L, int m,
                                                     double *x) {
    BCHUNK;
    if (!B.valid[c]) return;
    const int k = B.kcol[c];
    const double *y = B.y + static_cast<int64_t>(c) * m;
    double s = x[e];
    for (int i = 0; i < k; ++i) s += Z[static_cast<int64_t>(i) * L + e] * y[i];
    x[e] = s;
}

// ---------------------------------------------------------------- plain CG (FP64), every column

// r = b, p = b (x0 = 0); per column b.b.
__global__ __launch_bounds__(BLOCK) void kc_init(BCols B, const double *__restrict__ b, double *r, double *p) {
    BCHUNK;
    if (!B.valid[c]) {
        r[e] = 0.0;
        p[e] = 0.0;
        return;
    }
    const double v = b[e];
    r[e] = v;
    p[e] = v;
    double acc[1] = {v * v};
    seg_partial(acc, B);
}

__global__ __launch_bounds__(BLOCK) void kc_init_col(BCols B, int C) {
    const int c = wave_col(C);
    if (c < 0 || !B.valid[c]) return;
    const double bb = col_sum(B, c, 0);
    if (threadIdx.x % WAVE == 0) {
        B.bnorm[c] = sqrt(bb);
        B.rr64[c] = bb;
        B.est[c] = bb > 0.0 ? 1.0 : 0.0;
        B.cg_iters[c] = 0;
        B.cand[c] = 0;
        B.restart[c] = 0;
        if (!isfinite(bb)) {
            B.status[c] = KRR_ENONFINITE;
            B.valid[c] = 0;
            B.cg_active[c] = 0;
            return;
        }
        B.cg_active[c] = bb > 0.0 ? 1 : 0;
    }
}

__global__ __launch_bounds__(BLOCK) void kc_alpha(BCols B, const double *__restrict__ p,
                                                  const double *__restrict__ Ap) {
    BCHUNK;
    if (!B.cg_active[c]) return;
    double acc[1] = {p[e] * Ap[e]};
    seg_partial(acc, B);
}

__global__ __launch_bounds__(BLOCK) void kc_alpha_col(BCols B, int C) {
    const int c = wave_col(C);
    if (c < 0 || !B.cg_active[c]) return;
    const double pAp = col_sum(B, c, 0);
    if (threadIdx.x % WAVE == 0) {
        B.restart[c] = 0;
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            B.cg_active[c] = 0;
            B.status[c] = KRR_BREAKDOWN;
            B.cand[c] = 1;  // its true residual is still reported
        } else {
            B.alpha64[c] = B.rr64[c] / pAp;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void kc_update(BCols B, double *x, double *r, const double *__restrict__ p,
                                                   const double *__restrict__ Ap) {
    BCHUNK;
    if (!B.cg_active[c]) return;
    const double a = B.alpha64[c];
    x[e] += a * p[e];
    const double ri = r[e] - a * Ap[e];
    r[e] = ri;
    double acc[1] = {ri * ri};
    seg_partial(acc, B);
}

// A column whose recursive residual reaches the tolerance, or that reaches the
// iteration cap, stops and waits for its true-residual check.
__global__ __launch_bounds__(BLOCK) void kc_update_col(BCols B, int C, double tol2, int maxit) {
    const int c = wave_col(C);
    if (c < 0 || !B.cg_active[c]) return;
    const double rr = col_sum(B, c, 0);
    if (threadIdx.x % WAVE == 0) {
        B.beta64[c] = rr / B.rr64[c];
        B.rr64[c] = rr;
        const int it = B.cg_iters[c] + 1;
        B.cg_iters[c] = it;
        B.col_mvp64[c] += 1;
        const double bb = B.bnorm[c] * B.bnorm[c];
        if (!isfinite(rr)) {
            B.cg_active[c] = 0;
            B.status[c] = KRR_BREAKDOWN;
            B.cand[c] = 1;
        } else if (rr <= tol2 * bb || it >= maxit) {
            B.cg_active[c] = 0;
            B.cand[c] = 1;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void kc_pupdate(BCols B, const double *__restrict__ r, double *p) {
    BCHUNK;
    if (!B.cg_active[c]) return;
    p[e] = r[e] + B.beta64[c] * p[e];
}

// True residual r = b - K x of the columns to check.
__global__ __launch_bounds__(BLOCK) void kc_true(BCols B, const double *__restrict__ b,
                                                 const double *__restrict__ Kx, double *r) {
    BCHUNK;
    if (!B.cand[c]) return;
    const double v = b[e] - Kx[e];
    r[e] = v;
    double acc[1] = {v * v};
    seg_partial(acc, B);
}

// Accept a checked column (its true residual meets the tolerance, it broke
// down, or it reached the cap) or restart its CG from the true residual.
__global__ __launch_bounds__(BLOCK) void kc_true_col(BCols B, int C, double tol, int maxit) {
    const int c = wave_col(C);
    if (c < 0 || !B.cand[c]) return;
    const double rr = col_sum(B, c, 0);
    if (threadIdx.x % WAVE == 0) {
        B.cand[c] = 0;
        B.col_mvp64[c] += 1;
        const double bn = B.bnorm[c];
        const double est = bn > 0.0 ? sqrt(rr) / bn : 0.0;
        B.est[c] = est;
        if (B.status[c] != 0 || est <= tol || B.cg_iters[c] >= maxit || !isfinite(est)) return;
        B.rr64[c] = rr;
        B.restart[c] = 1;
        B.cg_active[c] = 1;
        B.col_cycles[c] += 1;
    }
}

__global__ __launch_bounds__(BLOCK) void kc_prestart(BCols B, const double *__restrict__ r, double *p) {
    BCHUNK;
    if (!B.restart[c]) return;
    p[e] = r[e];
}

// summary[0] = columns in their FGMRES cycle, [1] = non-finite right-hand
// sides, [2] = active plain-CG columns, [3] = plain-CG columns to check
__global__ void kb_summary(BCols B, int C) {
    __shared__ int sh[4][BLOCK];
    int v[4] = {0, 0, 0, 0};
    for (int c = threadIdx.x; c < C; c += BLOCK) {
        v[0] += B.in_cycle[c];
        v[1] += B.status[c] == KRR_ENONFINITE ? 1 : 0;
        v[2] += B.cg_active[c];
        v[3] += B.cand[c];
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        int t = 0;
        for (int i = 0; i < BLOCK; ++i) t += sh[threadIdx.x][i];
        B.summary[threadIdx.x] = t;
    }
}

__global__ void kb_fill_i(int *p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Gather system k's right-hand sides (original order, column-major, ld) into
// its sorted block (n_pad x Rp, zero padding and zero extra columns); scatter
// the solution back.
__global__ __launch_bounds__(BLOCK) void kb_gather(const int32_t *__restrict__ perm, int64_t n_pad, int nrhs, int Rp,
                                                   const double *__restrict__ Y, int64_t ld, double *dst) {
    const int64_t idx = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (idx >= n_pad * Rp) return;
    const int64_t i = idx % n_pad;
    const int r = static_cast<int>(idx / n_pad);
    const int32_t p = perm[i];
    dst[idx] = (r < nrhs && p >= 0) ? Y[p + static_cast<int64_t>(r) * ld] : 0.0;
}
__global__ __launch_bounds__(BLOCK) void kb_scatter(const int32_t *__restrict__ perm, int64_t n_pad, int nrhs,
                                                    const double *__restrict__ src, double *W, int64_t ld) {
    const int64_t idx = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (idx >= n_pad * nrhs) return;
    const int64_t i = idx % n_pad;
    const int r = static_cast<int>(idx / n_pad);
    const int32_t p = perm[i];
    if (p >= 0) W[p + static_cast<int64_t>(r) * ld] = src[idx];
}

struct Sys {
    Prepared P;
    int64_t base = 0;  // element offset of the system block
    double sigma = 0, gamma = 0, delta = 0;
    void *pscratch = nullptr;  // its batched-product scratch
};

struct BatchLayout {
    std::vector<Sys> sys;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    MSysB *d_sys_in = nullptr, *d_sys_out = nullptr;  // [nprob], grouped by dimension class
    MItem *d_items = nullptr;
    int nitems = 0;     // capacity: items at the smallest candidate tile count
    int64_t L = 0;
    int nchunks = 0, C = 0, Rp = 0;
    double *b = nullptr, *x = nullptr, *w = nullptr, *r = nullptr, *vin = nullptr, *V = nullptr, *Z = nullptr;
    float *z32 = nullptr, *r32 = nullptr, *p32 = nullptr, *Ap32 = nullptr;
    BCols B;
    size_t total = 0;
};

// Candidate column tiles per work item of a batched product (the autotuner
// times them once per dimension class and keeps the fastest).
constexpr int kTpsCands[] = {16, 32, 64, 128};
constexpr int kTpsMin = 16;

int64_t items_of(int ntiles, int tps, int nrb) {
    const int t = ntiles < tps ? ntiles : tps;
    return static_cast<int64_t>(ntiles) * ((ntiles + t - 1) / t) * nrb;
}

// m: restart length (0: plain CG, which keeps no basis)
BatchLayout carve_batch(void *ws, const krr_points *probs, int nprob, int nrhs, int m) {
    Carver cv(ws);
    BatchLayout L;
    L.Rp = (nrhs + 15) / 16 * 16;
    int64_t maxn = 1;
    L.sys.resize(nprob);
    const int nrb = L.Rp / 16;
    int64_t nitems = 0;
    for (int k = 0; k < nprob; ++k) {
        L.sys[k].P = carve_prepared(cv, probs[k].n, probs[k].d);
        L.sys[k].base = L.L;
        L.L += L.sys[k].P.n_pad * L.Rp;
        if (probs[k].n > maxn) maxn = probs[k].n;
        L.sys[k].pscratch = cv.take<char>(batched_product_scratch_bytes(L.sys[k].P, L.Rp, kTpsMin));
        nitems += items_of(L.sys[k].P.ntiles, kTpsMin, nrb);
    }
    L.nitems = static_cast<int>(nitems);
    L.temp_bytes = prep_temp_bytes(maxn);
    L.temp = cv.take<char>(L.temp_bytes);
    L.d_sys_in = cv.take<MSysB>(nprob);
    L.d_sys_out = cv.take<MSysB>(nprob);
    L.d_items = cv.take<MItem>(L.nitems);
    L.nchunks = static_cast<int>(L.L / BLOCK);
    L.C = nprob * L.Rp;
    const int64_t n = L.L;
    L.b = cv.take<double>(n);
    L.x = cv.take<double>(n);
    L.w = cv.take<double>(n);
    L.r = cv.take<double>(n);
    L.vin = cv.take<double>(n);
    if (m > 0) {
        L.V = cv.take<double>(static_cast<size_t>(m + 1) * n);
        L.Z = cv.take<double>(static_cast<size_t>(m) * n);
        L.z32 = cv.take<float>(n);
        L.r32 = cv.take<float>(n);
        L.p32 = cv.take<float>(n);
        L.Ap32 = cv.take<float>(n);
    }
    const int C = L.C;
    const int mm = m > 0 ? m : 1;
    BCols &B = L.B;
    B.rr = cv.take<float>(C);
    B.rr0 = cv.take<float>(C);
    B.thresh = cv.take<float>(C);
    B.alpha = cv.take<float>(C);
    B.beta = cv.take<float>(C);
    B.cg_active = cv.take<int>(C);
    B.cg_iters = cv.take<int>(C);
    B.bnorm = cv.take<double>(C);
    B.beta_o = cv.take<double>(C);
    B.est = cv.take<double>(C);
    B.wnorm0 = cv.take<double>(C);
    B.breakdown = cv.take<int>(C);
    B.in_cycle = cv.take<int>(C);
    B.kcol = cv.take<int>(C);
    B.valid = cv.take<int>(C);
    B.status = cv.take<int>(C);
    B.col_outer = cv.take<int>(C);
    B.col_inner = cv.take<int>(C);
    B.col_mvp64 = cv.take<int>(C);
    B.col_cycles = cv.take<int>(C);
    B.H = cv.take<double>(static_cast<size_t>(C) * mm * (mm + 1));
    B.cs = cv.take<double>(static_cast<size_t>(C) * mm);
    B.sn = cv.take<double>(static_cast<size_t>(C) * mm);
    B.g = cv.take<double>(static_cast<size_t>(C) * (mm + 1));
    B.y = cv.take<double>(static_cast<size_t>(C) * mm);
    B.hcol = cv.take<double>(static_cast<size_t>(C) * (mm + 2));
    B.gcoef = cv.take<double>(static_cast<size_t>(C) * (mm + 2));
    B.rr64 = cv.take<double>(C);
    B.alpha64 = cv.take<double>(C);
    B.beta64 = cv.take<double>(C);
    B.cand = cv.take<int>(C);
    B.restart = cv.take<int>(C);
    B.chunk_col = cv.take<int>(L.nchunks);
    B.col_chunk0 = cv.take<int>(C);
    B.col_nchunk = cv.take<int>(C);
    B.col_off = cv.take<int64_t>(C);
    B.pstride = mm + 2;
    B.partials = cv.take<double>(static_cast<size_t>(L.nchunks) * B.pstride);
    B.summary = cv.take<int>(4);
    L.total = cv.off + 256;
    return L;
}

double wall_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

size_t batch_workspace_bytes(const krr_points *probs, int nprob, int nrhs, int m) {
    return carve_batch(nullptr, probs, nprob, nrhs, m).total;
}

#define BH(expr)                                        \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return KRR_EHIP;          \
    } while (0)

namespace {

// Everything a batched solve sets up before it iterates: the carved layout,
// the column maps, the prepared systems with their gathered right-hand sides,
// and one batched product per dimension class in the inner precision and in
// FP64, with the work-item tile chosen by the autotuner.
struct BatchRun {
    BatchLayout L;
    std::vector<BatchedProduct> bp_in, bp_out;
    std::vector<int> class_tps;  // tuned column tiles per work item, per class
    int nprob = 0, nrhs = 0;
    double t_prep_ms = 0.0;

    hipError_t products(const void *Q, void *Yo, bool inner, ColGate gate, hipStream_t st) const {
        for (size_t c = 0; c < bp_in.size(); ++c)
            KRR_HIP(batched_product(inner ? bp_in[c] : bp_out[c], Q, Yo, inner ? 1 : 0, gate, st));
        return hipSuccess;
    }
};

// Work items of one class at `tps` column tiles per item, largest systems first.
void class_items(const BatchLayout &L, const std::vector<int> &order, int pos, int end, int tps, int nrb,
                 std::vector<MItem> &items) {
    for (int e = pos; e < end; ++e) {
        const Prepared &P = L.sys[order[e]].P;
        const int t = P.ntiles < tps ? P.ntiles : tps;
        const int splits = (P.ntiles + t - 1) / t;
        for (int bx = 0; bx < P.ntiles; ++bx)
            for (int by = 0; by < splits; ++by)
                for (int rb = 0; rb < nrb; ++rb) items.push_back(MItem{e - pos, bx, by, rb});
    }
}

int batch_setup(BatchRun &R, const krr_points *probs, int nprob, const double *sigma, const double *gamma, int nrhs,
                const double *const *Y, const int64_t *ldy, const SolverOpts &o, int m, void *ws, size_t ws_bytes,
                hipStream_t s) {
    const double t0 = wall_ms();
    R.nprob = nprob;
    R.nrhs = nrhs;
    R.L = carve_batch(nullptr, probs, nprob, nrhs, m);
    if (R.L.total > ws_bytes) return KRR_EWORKSPACE;
    R.L = carve_batch(ws, probs, nprob, nrhs, m);
    BatchLayout &L = R.L;
    const BCols &B = L.B;
    const int C = L.C, Rp = L.Rp;
    const int nb = L.nchunks;
    const int cb = (C + BLOCK - 1) / BLOCK;
    {
        std::vector<int> chunk_col(nb), col_chunk0(C), col_nchunk(C), valid(C);
        std::vector<int64_t> col_off(C);
        for (int k = 0; k < nprob; ++k) {
            const int64_t np = L.sys[k].P.n_pad;
            for (int r = 0; r < Rp; ++r) {
                const int c = k * Rp + r;
                col_off[c] = L.sys[k].base + r * np;
                col_chunk0[c] = static_cast<int>(col_off[c] / BLOCK);
                col_nchunk[c] = static_cast<int>(np / BLOCK);
                valid[c] = r < nrhs ? 1 : 0;
                for (int q = 0; q < col_nchunk[c]; ++q) chunk_col[col_chunk0[c] + q] = c;
            }
        }
        BH(hipMemcpyAsync(B.chunk_col, chunk_col.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
        BH(hipMemcpyAsync(B.col_chunk0, col_chunk0.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
        BH(hipMemcpyAsync(B.col_nchunk, col_nchunk.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
        BH(hipMemcpyAsync(B.col_off, col_off.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
        BH(hipMemcpyAsync(B.valid, valid.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
        BH(hipStreamSynchronize(s));  // host vectors go out of scope
    }
    int *zero_int[] = {B.kcol, B.in_cycle, B.cg_active, B.breakdown, B.status, B.col_outer, B.col_inner,
                       B.col_mvp64, B.col_cycles, B.cand, B.restart, B.cg_iters};
    for (int *p : zero_int) hipLaunchKernelGGL(kb_fill_i, dim3(cb), dim3(BLOCK), 0, s, p, C, 0);
    BH(fill_d(B.est, C, 0.0, s));

    // prepare every system; gather its right-hand sides; x = 0
    for (int k = 0; k < nprob; ++k) {
        Sys &S = L.sys[k];
        S.sigma = sigma[k];
        S.gamma = gamma[k];
        S.delta = o.delta >= 0 ? o.delta : (gamma[k] > 0 ? 10 * gamma[k] : 1e-3);
        BH(prepare_points(S.P, probs[k].x, sigma[k], L.temp, L.temp_bytes, s));
        int flag = 0;
        BH(hipMemcpyAsync(&flag, S.P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        BH(hipStreamSynchronize(s));
        if (flag & 1) return KRR_ENONFINITE;
        const int64_t ld = ldy ? ldy[k] : probs[k].n;
        const int64_t tot = S.P.n_pad * Rp;
        hipLaunchKernelGGL(kb_gather, dim3((tot + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, S.P.perm, S.P.n_pad, nrhs,
                           Rp, Y[k], ld, L.b + S.base);
    }
    BH(fill_d(L.x, L.L, 0.0, s));
    const int inner_prec = (o.inner_prec == KRR_BF16) ? KRR_BF16 : KRR_FP32;

    // systems grouped by compiled dimension, largest first inside a class
    std::vector<int> order(nprob);
    for (int k = 0; k < nprob; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        const int da = L.sys[a].P.dpad, db = L.sys[b].P.dpad;
        return da != db ? da < db : L.sys[a].P.n > L.sys[b].P.n;
    });
    const int nrb = Rp / 16;
    std::vector<MSysB> hin(nprob), hout(nprob);
    std::vector<MItem> items;
    items.reserve(L.nitems);
    auto fill_class = [&](int pos, int end, int tps) {
        for (int e = pos; e < end; ++e) {
            const Sys &S = L.sys[order[e]];
            fill_msys(hin[e], S.P, inner_prec, Rp, S.pscratch, S.base, S.delta, S.gamma, tps);
            fill_msys(hout[e], S.P, KRR_FP64, Rp, S.pscratch, S.base, S.delta, S.gamma, tps);
            hin[e].col0 = hout[e].col0 = order[e] * Rp;
        }
    };
    // KRR_BATCH_TPS=k fixes the column tiles per work item
    const char *ftps = std::getenv("KRR_BATCH_TPS");
    const int forced = ftps ? std::max(std::atoi(ftps), kTpsMin) : 0;  // the scratch holds kTpsMin tiles and up
    // the tuned product: the inner one of a flexible solve (on the zeroed FP32
    // CG direction), the FP64 one of a plain CG solve (on the right-hand sides)
    const bool tune_inner = m > 0;
    if (tune_inner) BH(zero_bytes(L.p32, L.L * static_cast<int64_t>(sizeof(float)), s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int pos = 0;
    while (pos < nprob) {
        const int dp = L.sys[order[pos]].P.dpad;
        int end = pos;
        int class_tiles = 0;
        double pairs = 0.0;
        int64_t me = 0;
        while (end < nprob && L.sys[order[end]].P.dpad == dp) {
            const Prepared &P = L.sys[order[end]].P;
            class_tiles += P.ntiles;
            pairs += static_cast<double>(P.n) * static_cast<double>(P.n);
            me = std::max<int64_t>(me, P.n_pad * 16 * nrb);
            ++end;
        }
        BatchedProduct bi, bo;
        bi.dpad = bo.dpad = dp;
        bi.prec = inner_prec;
        bo.prec = KRR_FP64;
        bi.nrhs = bo.nrhs = Rp;
        bi.d_sys = L.d_sys_in + pos;
        bo.d_sys = L.d_sys_out + pos;
        bi.d_items = bo.d_items = L.d_items + items.size();
        bi.nsys = bo.nsys = end - pos;
        bi.max_elems = bo.max_elems = me;
        bi.pairs = bo.pairs = pairs;
        // the tile: forced, cached, or timed now on this class (inner precision,
        // every column live) and cached for the process and KRR_TUNE_CACHE
        int tps = forced > 0 ? forced : 0;
        const int tune_prec = tune_inner ? inner_prec : KRR_FP64;
        if (tps == 0 && !tune_lookup(64 + tune_prec, dp, class_tiles * nrb, &tps)) {
            if (!e0) {
                BH(hipEventCreate(&e0));
                BH(hipEventCreate(&e1));
            }
            float best_ms = 1e30f;
            for (int cand : kTpsCands) {
                std::vector<MItem> ci;
                class_items(L, order, pos, end, cand, nrb, ci);
                fill_class(pos, end, cand);
                BatchedProduct bt = tune_inner ? bi : bo;
                const void *tq = tune_inner ? static_cast<const void *>(L.p32) : static_cast<const void *>(L.b);
                void *ty = tune_inner ? static_cast<void *>(L.Ap32) : static_cast<void *>(L.w);
                BH(hipMemcpyAsync(bt.d_sys, (tune_inner ? hin : hout).data() + pos, sizeof(MSysB) * (end - pos),
                                  hipMemcpyHostToDevice, s));
                BH(hipMemcpyAsync(bt.d_items, ci.data(), sizeof(MItem) * ci.size(), hipMemcpyHostToDevice, s));
                bt.nitems = static_cast<int>(ci.size());
                profile_suspend(true);
                hipError_t err = batched_product(bt, tq, ty, 1, ColGate{}, s);  // warm
                if (err == hipSuccess) err = hipEventRecord(e0, s);
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) err = batched_product(bt, tq, ty, 1, ColGate{}, s);
                if (err == hipSuccess) err = hipEventRecord(e1, s);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                profile_suspend(false);
                float ms = 0.f;
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                if (err != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return KRR_EHIP;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    tps = cand;
                }
            }
            tune_store(64 + tune_prec, dp, class_tiles * nrb, tps);
        }
        R.class_tps.push_back(tps);
        class_items(L, order, pos, end, tps, nrb, items);
        fill_class(pos, end, tps);
        bi.nitems = bo.nitems = static_cast<int>((L.d_items + items.size()) - bi.d_items);
        R.bp_in.push_back(bi);
        R.bp_out.push_back(bo);
        pos = end;
    }
    if (e0) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    if (static_cast<int>(items.size()) > L.nitems) return KRR_EHIP;  // cannot happen: capacity at the smallest tile
    BH(hipMemcpyAsync(L.d_sys_in, hin.data(), sizeof(MSysB) * nprob, hipMemcpyHostToDevice, s));
    BH(hipMemcpyAsync(L.d_sys_out, hout.data(), sizeof(MSysB) * nprob, hipMemcpyHostToDevice, s));
    BH(hipMemcpyAsync(L.d_items, items.data(), sizeof(MItem) * items.size(), hipMemcpyHostToDevice, s));
    BH(hipStreamSynchronize(s));
    R.t_prep_ms = wall_ms() - t0;
    return KRR_OK;
}

// Per-column results into infos; returns the call's status: KRR_ENONFINITE if
// any right-hand side was not finite (the other columns are still solved),
// else the worst column status.
int batch_report(const BatchRun &R, double tol, int inner_prec, int steps, double t_total_ms, krr_info *infos,
                 hipStream_t s) {
    const BatchLayout &L = R.L;
    const int C = L.C, Rp = L.Rp;
    std::vector<double> est(C);
    std::vector<int> st(C), outer(C), inner(C), mvp(C), cyc(C), iters(C);
    BH(hipMemcpyAsync(est.data(), L.B.est, sizeof(double) * C, hipMemcpyDeviceToHost, s));
    BH(hipMemcpyAsync(st.data(), L.B.status, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    BH(hipMemcpyAsync(outer.data(), L.B.col_outer, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    BH(hipMemcpyAsync(inner.data(), L.B.col_inner, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    BH(hipMemcpyAsync(mvp.data(), L.B.col_mvp64, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    BH(hipMemcpyAsync(cyc.data(), L.B.col_cycles, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    BH(hipMemcpyAsync(iters.data(), L.B.cg_iters, sizeof(int) * C, hipMemcpyDeviceToHost, s));
    BH(hipStreamSynchronize(s));
    int worst = KRR_OK;
    bool nonfinite = false;
    for (int k = 0; k < R.nprob; ++k)
        for (int r = 0; r < R.nrhs; ++r) {
            const int c = k * Rp + r;
            int status = st[c] != 0 ? st[c] : (est[c] <= tol ? KRR_OK : KRR_NOT_CONVERGED);
            if (status == KRR_ENONFINITE) nonfinite = true;
            else if (status > worst) worst = status;
            if (!infos) continue;
            krr_info &I = infos[static_cast<size_t>(k) * R.nrhs + r];
            std::memset(&I, 0, sizeof(I));
            I.status = status;
            const bool cg = inner_prec < 0;
            I.outer_iters = cg ? iters[c] : outer[c];
            I.inner_iters = cg ? 0 : inner[c];
            I.cycles = cg ? cyc[c] + 1 : cyc[c];
            I.mvp64 = mvp[c];
            if (!cg) {
                if (inner_prec == KRR_BF16) I.mvp16 = inner[c];
                else I.mvp32 = inner[c];
            }
            I.relres_true = status == KRR_ENONFINITE ? NAN : est[c];
            I.relres_est = I.relres_true;
            I.t_total_ms = t_total_ms;
            I.t_prep_ms = R.t_prep_ms;
            I.batch_steps = steps;
            I.batch_tiles = R.class_tps.empty() ? 0 : R.class_tps[0];
        }
    return nonfinite ? KRR_ENONFINITE : worst;
}

void scatter_solutions(const BatchRun &R, const krr_points *probs, double *const *W, const int64_t *ldy,
                       hipStream_t s) {
    const BatchLayout &L = R.L;
    for (int k = 0; k < R.nprob; ++k) {
        const Sys &S = L.sys[k];
        const int64_t ld = ldy ? ldy[k] : probs[k].n;
        const int64_t tot = S.P.n_pad * R.nrhs;
        hipLaunchKernelGGL(kb_scatter, dim3((tot + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, S.P.perm, S.P.n_pad,
                           R.nrhs, L.x + S.base, W[k], ld);
    }
}

}  // namespace

// The batched mixed-precision FGMRES (inner CG in o.inner_prec: FP32 or BF16
// products, FP32 vectors; outer FP64; Gram-Schmidt o.gs).  Y, W, ldy: host
// arrays of device pointers / leading dimensions.  infos: nprob * nrhs entries
// (may be null).  Each outer step (the inner CG, the outer product, the
// Gram-Schmidt passes, the normalisation and the Givens step of every column)
// is one HIP graph per step index, recorded at its first use; the host reads a
// 16-byte summary every o.cg_check steps and at cycle ends.
int batched_fgmres(const krr_points *probs, int nprob, const double *sigma, const double *gamma, int nrhs,
                   const double *const *Y, const int64_t *ldy, double *const *W, const SolverOpts &o,
                   krr_info *infos, void *ws, size_t ws_bytes, hipStream_t s) {
    const double t0 = wall_ms();
    if (o.inner != KRR_INNER_NONE && o.inner_prec == KRR_FP64) return KRR_EUNSUPPORTED;  // routed by the caller
    const int m = o.restart_m;
    BatchRun R;
    int rc = batch_setup(R, probs, nprob, sigma, gamma, nrhs, Y, ldy, o, m, ws, ws_bytes, s);
    if (rc != KRR_OK) return rc;
    const BatchLayout &L = R.L;
    const BCols &B = L.B;
    const int C = L.C;
    const int64_t LL = L.L;
    const int nb = L.nchunks;
    const int cb = (C + BLOCK - 1) / BLOCK;
    const int ccb = (C + BLOCK / WAVE - 1) / (BLOCK / WAVE);  // one wave per column
    const int inner_prec = (o.inner_prec == KRR_BF16) ? KRR_BF16 : KRR_FP32;
    const int check = o.cg_check > 0 ? o.cg_check : 16;

    // Products run only on the columns that use them: the inner CG's on columns
    // in their cycle with an active CG, the Arnoldi step's on columns in their
    // cycle, the cycle-end residual's on columns that took a step this cycle.
    const ColGate gate_inner{B.in_cycle, B.cg_active}, gate_arnoldi{B.in_cycle, nullptr},
        gate_cycle_end{B.kcol, nullptr};

    // one outer step j on fixed buffers: the inner CG (V_j -> z32 -> Z_j), the
    // outer product w = K Z_j, Gram-Schmidt, v_{j+1}, Givens
    const double tol2 = o.inner_tol * o.inner_tol;
    auto step_seq = [&](int j, hipStream_t st) -> hipError_t {
        double *Vj = L.V + static_cast<int64_t>(j) * LL;
        double *Zj = L.Z + static_cast<int64_t>(j) * LL;
        if (o.inner == KRR_INNER_NONE) {
            hipLaunchKernelGGL(kb_copy, dim3(nb), dim3(BLOCK), 0, st, B, Vj, Zj);
        } else {
            hipLaunchKernelGGL(kb_copy, dim3(nb), dim3(BLOCK), 0, st, B, Vj, L.vin);
            hipLaunchKernelGGL(kb_cg_init, dim3(nb), dim3(BLOCK), 0, st, B, L.vin, L.z32, L.r32, L.p32);
            hipLaunchKernelGGL(kb_cg_init_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, tol2, o.inner_maxit);
            for (int it = 0; it < o.inner_maxit; ++it) {
                KRR_HIP(R.products(L.p32, L.Ap32, true, gate_inner, st));
                hipLaunchKernelGGL(kb_cg_alpha, dim3(nb), dim3(BLOCK), 0, st, B, L.p32, L.Ap32);
                hipLaunchKernelGGL(kb_cg_alpha_col, dim3(ccb), dim3(BLOCK), 0, st, B, C);
                hipLaunchKernelGGL(kb_cg_update, dim3(nb), dim3(BLOCK), 0, st, B, L.z32, L.r32, L.p32, L.Ap32);
                hipLaunchKernelGGL(kb_cg_update_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, o.inner_maxit);
                hipLaunchKernelGGL(kb_cg_pupdate, dim3(nb), dim3(BLOCK), 0, st, B, L.r32, L.p32);
            }
            hipLaunchKernelGGL(kb_cast_z, dim3(nb), dim3(BLOCK), 0, st, B, L.z32, Zj);
        }
        KRR_HIP(R.products(Zj, L.w, false, gate_arnoldi, st));
        if (o.gs == KRR_GS_CGS2) {
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(kb_gs_dot, dim3(nb), dim3(BLOCK), 0, st, B, L.w, L.V, LL, j, pass == 0 ? 1 : 0);
                hipLaunchKernelGGL(kb_gs_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, j, pass, m);
                hipLaunchKernelGGL(kb_gs_update, dim3(nb), dim3(BLOCK), 0, st, B, L.w, L.V, LL, j, m);
            }
            hipLaunchKernelGGL(kb_wsq, dim3(nb), dim3(BLOCK), 0, st, B, L.w);
            hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, 2, j + 1, m);
        } else {
            hipLaunchKernelGGL(kb_mgs_first, dim3(nb), dim3(BLOCK), 0, st, B, L.w, L.V);
            hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, 0, 0, m);
            for (int i = 0; i < j; ++i) {
                hipLaunchKernelGGL(kb_mgs_step, dim3(nb), dim3(BLOCK), 0, st, B, L.w, L.V + i * LL,
                                   L.V + (i + 1) * LL, i, m);
                hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, 1, i + 1, m);
            }
            hipLaunchKernelGGL(kb_mgs_last, dim3(nb), dim3(BLOCK), 0, st, B, L.w, Vj, j, m);
            hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, 2, j + 1, m);
        }
        // normalise before the Givens step decides whether the column leaves its cycle
        hipLaunchKernelGGL(kb_normalize, dim3(nb), dim3(BLOCK), 0, st, B, L.w, L.V + (j + 1) * LL, j, m);
        hipLaunchKernelGGL(kb_givens, dim3(cb), dim3(BLOCK), 0, st, B, C, j, m, o.tol);
        return hipGetLastError();
    };

    // KRR_NO_GRAPH=1 runs the same step sequences eagerly (used to check that
    // the graph replays give bit-identical results)
    const char *nog = std::getenv("KRR_NO_GRAPH");
    const bool use_graph = !(nog && nog[0] == '1');
    hipStream_t gs = nullptr;
    std::vector<hipGraphExec_t> gexec(m, nullptr);
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    auto cleanup = [&]() {
        for (auto &g : gexec)
            if (g) (void)hipGraphExecDestroy(g);
        if (gs) (void)hipStreamDestroy(gs);
        if (ev_a) (void)hipEventDestroy(ev_a);
        if (ev_b) (void)hipEventDestroy(ev_b);
    };
    if (use_graph && (hipStreamCreateWithFlags(&gs, hipStreamNonBlocking) != hipSuccess ||
                      hipEventCreate(&ev_a) != hipSuccess || hipEventCreate(&ev_b) != hipSuccess)) {
        cleanup();
        return KRR_EHIP;
    }
    auto run_step = [&](int j) -> hipError_t {
        if (!use_graph) return step_seq(j, s);
        if (!gexec[j]) {
            hipGraph_t graph = nullptr;
            profile_suspend(true);  // no timing events inside the recorded graph
            hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) e = step_seq(j, gs);
            hipError_t e2 = hipStreamEndCapture(gs, &graph);
            profile_suspend(false);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&gexec[j], graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            KRR_HIP(e);
        }
        KRR_HIP(hipEventRecord(ev_a, s));
        KRR_HIP(hipStreamWaitEvent(gs, ev_a, 0));
        KRR_HIP(hipGraphLaunch(gexec[j], gs));
        KRR_HIP(hipEventRecord(ev_b, gs));
        return hipStreamWaitEvent(s, ev_b, 0);
    };

    int host[4] = {0, 0, 0, 0};
    auto read_summary = [&]() -> hipError_t {
        hipLaunchKernelGGL(kb_summary, dim3(1), dim3(BLOCK), 0, s, B, C);
        KRR_HIP(hipMemcpyAsync(host, B.summary, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
        return hipStreamSynchronize(s);
    };
#define BHC(expr)                          \
    do {                                   \
        if ((expr) != hipSuccess) {        \
            cleanup();                     \
            return KRR_EHIP;               \
        }                                  \
    } while (0)

    hipLaunchKernelGGL(kb_residual, dim3(nb), dim3(BLOCK), 0, s, B, L.b, nullptr, L.r);
    hipLaunchKernelGGL(kb_residual_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, 0, m, o.tol);
    BHC(read_summary());
    int steps = 0, cycles = 0;
    while (host[0] > 0 && steps < o.max_outer) {
        hipLaunchKernelGGL(kb_first_basis, dim3(nb), dim3(BLOCK), 0, s, B, L.r, L.V);
        for (int j = 0; j < m && steps < o.max_outer; ++j) {
            BHC(run_step(j));
            ++steps;
            if ((j + 1) % check == 0 || j + 1 == m || steps == o.max_outer) {
                BHC(read_summary());
                if (progress_every() && steps / progress_every() != (steps - check) / progress_every())
                    std::fprintf(stderr, "krr batched fgmres: outer %d cycle %d columns in their cycle %d of %d\n",
                                 steps, cycles + 1, host[0], nprob * nrhs);
                if (host[0] == 0) break;
            }
        }
        // x += Z y per column, then the true residual restarts the unconverged ones
        hipLaunchKernelGGL(kb_backsolve, dim3(cb), dim3(BLOCK), 0, s, B, C, m);
        hipLaunchKernelGGL(kb_update_x, dim3(nb), dim3(BLOCK), 0, s, B, L.Z, LL, m, L.x);
        ++cycles;
        BHC(R.products(L.x, L.w, false, gate_cycle_end, s));
        hipLaunchKernelGGL(kb_residual, dim3(nb), dim3(BLOCK), 0, s, B, L.b, L.w, L.r);
        hipLaunchKernelGGL(kb_residual_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, 1, m, o.tol);
        BHC(read_summary());
    }
#undef BHC
    scatter_solutions(R, probs, W, ldy, s);
    const int result = batch_report(R, o.tol, inner_prec, steps, wall_ms() - t0, infos, s);
    cleanup();
    return result;
}

// Plain FP64 CG over every (system, column) pair at once (the comparator of
// the batched mixed solve): FP64 multi-RHS products gated per column,
// segmented reductions, per-column step lengths; a column whose recursive
// residual reaches the tolerance is checked with its true residual and either
// accepted or restarted from it, while the others keep iterating.  The host
// reads a 16-byte summary every o.cg_check iterations.
int batched_cg64(const krr_points *probs, int nprob, const double *sigma, const double *gamma, int nrhs,
                 const double *const *Y, const int64_t *ldy, double *const *W, const SolverOpts &o, krr_info *infos,
                 void *ws, size_t ws_bytes, hipStream_t s) {
    const double t0 = wall_ms();
    BatchRun R;
    int rc = batch_setup(R, probs, nprob, sigma, gamma, nrhs, Y, ldy, o, 0, ws, ws_bytes, s);
    if (rc != KRR_OK) return rc;
    const BatchLayout &L = R.L;
    const BCols &B = L.B;
    const int C = L.C;
    const int nb = L.nchunks;
    const int ccb = (C + BLOCK / WAVE - 1) / (BLOCK / WAVE);
    const int check = o.cg_check > 0 ? o.cg_check : 16;
    double *p = L.vin, *Ap = L.w;
    const ColGate gate_active{B.cg_active, nullptr}, gate_cand{B.cand, nullptr};
    const double tol2 = o.tol * o.tol;

    int host[4] = {0, 0, 0, 0};
    auto read_summary = [&]() -> hipError_t {
        hipLaunchKernelGGL(kb_summary, dim3(1), dim3(BLOCK), 0, s, B, C);
        KRR_HIP(hipMemcpyAsync(host, B.summary, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
        return hipStreamSynchronize(s);
    };
    hipLaunchKernelGGL(kc_init, dim3(nb), dim3(BLOCK), 0, s, B, L.b, L.r, p);
    hipLaunchKernelGGL(kc_init_col, dim3(ccb), dim3(BLOCK), 0, s, B, C);
    BH(read_summary());
    int iters = 0;
    while (host[2] > 0 || host[3] > 0) {
        if (host[2] > 0) {
            for (int k = 0; k < check; ++k) {
                BH(R.products(p, Ap, false, gate_active, s));
                hipLaunchKernelGGL(kc_alpha, dim3(nb), dim3(BLOCK), 0, s, B, p, Ap);
                hipLaunchKernelGGL(kc_alpha_col, dim3(ccb), dim3(BLOCK), 0, s, B, C);
                hipLaunchKernelGGL(kc_update, dim3(nb), dim3(BLOCK), 0, s, B, L.x, L.r, p, Ap);
                hipLaunchKernelGGL(kc_update_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, tol2, o.max_outer);
                hipLaunchKernelGGL(kc_pupdate, dim3(nb), dim3(BLOCK), 0, s, B, L.r, p);
            }
            iters += check;
            BH(read_summary());
            if (progress_every() && iters / progress_every() != (iters - check) / progress_every())
                std::fprintf(stderr, "krr batched cg64: iteration %d active columns %d of %d\n", iters, host[2],
                             nprob * nrhs);
        }
        if (host[3] > 0) {
            // true residuals of the columns that stopped; accept or restart
            BH(R.products(L.x, Ap, false, gate_cand, s));
            hipLaunchKernelGGL(kc_true, dim3(nb), dim3(BLOCK), 0, s, B, L.b, Ap, L.r);
            hipLaunchKernelGGL(kc_true_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, o.tol, o.max_outer);
            hipLaunchKernelGGL(kc_prestart, dim3(nb), dim3(BLOCK), 0, s, B, L.r, p);
            BH(read_summary());
        }
    }
    scatter_solutions(R, probs, W, ldy, s);
    return batch_report(R, o.tol, -1, iters, wall_ms() - t0, infos, s);
}

}  // namespace krr
