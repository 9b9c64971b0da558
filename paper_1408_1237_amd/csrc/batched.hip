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
    // CG
    float *rr, *rr0, *thresh, *alpha, *beta;
    int *cg_active, *cg_iters;
    // FGMRES
    double *bnorm, *beta_o, *est, *wnorm0;
    int *breakdown, *in_cycle, *kcol, *nonfinite, *valid;
    double *H, *cs, *sn, *g, *y, *hcol;  // C x (m+1) x m, C x m, C x m, C x (m+1), C x m, C x (m+2)
    int *chunk_col;    // [nchunks]
    int *col_chunk0;   // [C]
    int *col_nchunk;   // [C]
    int64_t *col_off;  // [C] element offset of the column
    double *partials;  // [nchunks * 2]
    int *summary;        // [4]: columns in cycle, columns active
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
        for (int k = 0; k < NV; ++k) B.partials[static_cast<int64_t>(blockIdx.x) * 2 + k] = v[k];
}

// Column of this wave (-1 past the last column).
__device__ __forceinline__ int wave_col(int C) {
    const int c = blockIdx.x * (BLOCK / WAVE) + static_cast<int>(threadIdx.x) / WAVE;
    return c < C ? c : -1;
}

// The column's totals, in every lane (lane l adds chunks l, l + 64, ...; then a
// fixed butterfly).  Called by all lanes of the wave.
template <int NV>
__device__ __forceinline__ void col_total(const BCols &B, int c, double (&v)[NV]) {
    const int c0 = B.col_chunk0[c], nc = B.col_nchunk[c];
    const int lane = static_cast<int>(threadIdx.x) % WAVE;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int q = lane; q < nc; q += WAVE) s += B.partials[static_cast<int64_t>(c0 + q) * 2 + k];
        v[k] = bwave_sum(s);
    }
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

__global__ __launch_bounds__(BLOCK) void kb_residual_col(BCols B, int C, int cycle_end, int m, double tol) {
    const int c = wave_col(C);
    if (c < 0 || !B.valid[c] || (cycle_end && B.kcol[c] == 0)) return;
    double acc[2];
    col_total(B, c, acc);
    if (threadIdx.x % WAVE == 0) {
        const double beta = sqrt(acc[0]), bn = sqrt(acc[1]);
        B.beta_o[c] = beta;
        B.bnorm[c] = bn;
        const double est = bn > 0.0 ? beta / bn : 0.0;
        B.est[c] = est;
        B.nonfinite[c] = isfinite(est) ? 0 : 1;
        B.in_cycle[c] = (est > tol && isfinite(est)) ? 1 : 0;
        B.kcol[c] = 0;
        B.breakdown[c] = 0;
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

__global__ __launch_bounds__(BLOCK) void kb_cast_z(BCols B, const float *__restrict__ z, double *Zj) {
    BCHUNK;
    if (!B.in_cycle[c]) return;
    Zj[e] = static_cast<double>(z[e]);
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

// Givens step of every column in its cycle (one thread per column); a column
// leaves the cycle on convergence of its estimate, on breakdown or non-finite.
__global__ void kb_givens(BCols B, int C, int j, int m, double tol) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C || !B.in_cycle[c]) return;
    const double *hc = B.hcol + static_cast<int64_t>(c) * (m + 2);
    double *col = B.H + (static_cast<int64_t>(c) * m + j) * (m + 1);
    double *cs = B.cs + static_cast<int64_t>(c) * m, *sn = B.sn + static_cast<int64_t>(c) * m;
    double *g = B.g + static_cast<int64_t>(c) * (m + 1);
    for (int i = 0; i <= j + 1; ++i) col[i] = hc[i];
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double rho = sqrt(a * a + b * b);
    cs[j] = a / rho;
    sn[j] = b / rho;
    col[j] = rho;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const double est = fabs(g[j + 1]) / B.bnorm[c];
    B.est[c] = est;
    B.kcol[c] = j + 1;
    const int brk = (hc[j + 1] > 1e-14 * B.wnorm0[c]) ? 0 : 1;
    B.breakdown[c] = brk;
    if (!isfinite(est)) {
        B.nonfinite[c] = 1;
        B.kcol[c] = j;
        B.in_cycle[c] = 0;
    } else if (brk || est <= tol) {
        B.in_cycle[c] = 0;
    }
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

// summary[0] = columns in their cycle, summary[1] = columns with a non-finite value
__global__ void kb_summary(BCols B, int C) {
    __shared__ int s0[BLOCK], s1[BLOCK];
    int a = 0, b = 0;
    for (int c = threadIdx.x; c < C; c += BLOCK) {
        a += B.in_cycle[c];
        b += B.nonfinite[c];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ta = 0, tb = 0;
        for (int t = 0; t < BLOCK; ++t) {
            ta += s0[t];
            tb += s1[t];
        }
        B.summary[0] = ta;
        B.summary[1] = tb;
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
    int nitems = 0;
    int64_t L = 0;
    int nchunks = 0, C = 0, Rp = 0;
    double *b = nullptr, *x = nullptr, *w = nullptr, *r = nullptr, *vin = nullptr, *V = nullptr, *Z = nullptr;
    float *z32 = nullptr, *r32 = nullptr, *p32 = nullptr, *Ap32 = nullptr;
    BCols B;
    size_t total = 0;
};

BatchLayout carve_batch(void *ws, const krr_points *probs, int nprob, int nrhs, int m) {
    Carver cv(ws);
    BatchLayout L;
    L.Rp = (nrhs + 15) / 16 * 16;
    int64_t maxn = 1;
    L.sys.resize(nprob);
    const int nrb = L.Rp / 16;
    for (int k = 0; k < nprob; ++k) {
        L.sys[k].P = carve_prepared(cv, probs[k].n, probs[k].d);
        L.sys[k].base = L.L;
        L.L += L.sys[k].P.n_pad * L.Rp;
        if (probs[k].n > maxn) maxn = probs[k].n;
        L.sys[k].pscratch = cv.take<char>(batched_product_scratch_bytes(L.sys[k].P, L.Rp));
        const int splits = (L.sys[k].P.ntiles + BATCH_TPS - 1) / BATCH_TPS;
        L.nitems += L.sys[k].P.ntiles * splits * nrb;
    }
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
    L.V = cv.take<double>(static_cast<size_t>(m + 1) * n);
    L.Z = cv.take<double>(static_cast<size_t>(m) * n);
    L.z32 = cv.take<float>(n);
    L.r32 = cv.take<float>(n);
    L.p32 = cv.take<float>(n);
    L.Ap32 = cv.take<float>(n);
    const int C = L.C;
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
    B.nonfinite = cv.take<int>(C);
    B.valid = cv.take<int>(C);
    B.H = cv.take<double>(static_cast<size_t>(C) * m * (m + 1));
    B.cs = cv.take<double>(static_cast<size_t>(C) * m);
    B.sn = cv.take<double>(static_cast<size_t>(C) * m);
    B.g = cv.take<double>(static_cast<size_t>(C) * (m + 1));
    B.y = cv.take<double>(static_cast<size_t>(C) * m);
    B.hcol = cv.take<double>(static_cast<size_t>(C) * (m + 2));
    B.chunk_col = cv.take<int>(L.nchunks);
    B.col_chunk0 = cv.take<int>(C);
    B.col_nchunk = cv.take<int>(C);
    B.col_off = cv.take<int64_t>(C);
    B.partials = cv.take<double>(static_cast<size_t>(L.nchunks) * 2);
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

// The batched mixed-precision FGMRES (inner CG in o.inner_prec: FP32 or BF16
// products, FP32 vectors; outer FP64).  Y, W, ldy: host arrays of device
// pointers / leading dimensions.  infos: nprob * nrhs entries (may be null).
int batched_fgmres(const krr_points *probs, int nprob, const double *sigma, const double *gamma, int nrhs,
                   const double *const *Y, const int64_t *ldy, double *const *W, const SolverOpts &o,
                   krr_info *infos, void *ws, size_t ws_bytes, hipStream_t s) {
    const double t0 = wall_ms();
    const int m = o.restart_m;
    BatchLayout L = carve_batch(nullptr, probs, nprob, nrhs, m);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve_batch(ws, probs, nprob, nrhs, m);
    const BCols &B = L.B;
    const int C = L.C, Rp = L.Rp;
    const int64_t LL = L.L;
    const int nb = L.nchunks;
    const int cb = (C + BLOCK - 1) / BLOCK;
    const int ccb = (C + BLOCK / WAVE - 1) / (BLOCK / WAVE);  // one wave per column

    // host-built chunk and column maps
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
    hipLaunchKernelGGL(kb_fill_i, dim3(cb), dim3(BLOCK), 0, s, B.nonfinite, C, 0);
    hipLaunchKernelGGL(kb_fill_i, dim3(cb), dim3(BLOCK), 0, s, B.kcol, C, 0);
    hipLaunchKernelGGL(kb_fill_i, dim3(cb), dim3(BLOCK), 0, s, B.in_cycle, C, 0);
    hipLaunchKernelGGL(kb_fill_i, dim3(cb), dim3(BLOCK), 0, s, B.cg_active, C, 0);
    hipLaunchKernelGGL(kb_fill_i, dim3(cb), dim3(BLOCK), 0, s, B.breakdown, C, 0);

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
    BH(fill_d(L.x, LL, 0.0, s));
    const int inner_prec = (o.inner_prec == KRR_BF16) ? KRR_BF16 : KRR_FP32;

    // Batched products: one launch (prescale, product, finish) per dimension
    // class and precision covers every system of that dimension.
    std::vector<BatchedProduct> bp_in, bp_out;
    {
        std::vector<int> order(nprob);
        for (int k = 0; k < nprob; ++k) order[k] = k;
        // group by compiled dimension, largest systems first inside a group
        std::sort(order.begin(), order.end(), [&](int a, int b) {
            const int da = L.sys[a].P.dpad, db = L.sys[b].P.dpad;
            return da != db ? da < db : L.sys[a].P.n > L.sys[b].P.n;
        });
        std::vector<MSysB> hin(nprob), hout(nprob);
        std::vector<MItem> items;
        items.reserve(L.nitems);
        const int nrb = Rp / 16;
        int pos = 0;
        while (pos < nprob) {
            const int dp = L.sys[order[pos]].P.dpad;
            int end = pos;
            BatchedProduct bi, bo;
            bi.dpad = bo.dpad = dp;
            bi.prec = inner_prec;
            bo.prec = KRR_FP64;
            bi.nrhs = bo.nrhs = Rp;
            bi.d_sys = L.d_sys_in + pos;
            bo.d_sys = L.d_sys_out + pos;
            bi.d_items = bo.d_items = L.d_items + items.size();
            while (end < nprob && L.sys[order[end]].P.dpad == dp) {
                const Sys &S = L.sys[order[end]];
                const int local = end - pos;
                fill_msys(hin[end], S.P, inner_prec, Rp, S.pscratch, S.base, S.delta, S.gamma);
                fill_msys(hout[end], S.P, KRR_FP64, Rp, S.pscratch, S.base, S.delta, S.gamma);
                hin[end].col0 = hout[end].col0 = order[end] * Rp;
                for (int bx = 0; bx < S.P.ntiles; ++bx)
                    for (int by = 0; by < hin[end].a.splits; ++by)
                        for (int rb = 0; rb < nrb; ++rb) items.push_back(MItem{local, bx, by, rb});
                const int64_t me = S.P.n_pad * 16 * nrb;
                bi.max_elems = bo.max_elems = std::max<int64_t>(bi.max_elems, me);
                bi.max_rows = bo.max_rows = std::max<int64_t>(bi.max_rows, S.P.n_pad * Rp);
                bi.pairs += static_cast<double>(S.P.n) * static_cast<double>(S.P.n);
                ++end;
            }
            bi.nsys = bo.nsys = end - pos;
            bi.nitems = bo.nitems = static_cast<int>((L.d_items + items.size()) - bi.d_items);
            bo.pairs = bi.pairs;
            bp_in.push_back(bi);
            bp_out.push_back(bo);
            pos = end;
        }
        BH(hipMemcpyAsync(L.d_sys_in, hin.data(), sizeof(MSysB) * nprob, hipMemcpyHostToDevice, s));
        BH(hipMemcpyAsync(L.d_sys_out, hout.data(), sizeof(MSysB) * nprob, hipMemcpyHostToDevice, s));
        BH(hipMemcpyAsync(L.d_items, items.data(), sizeof(MItem) * items.size(), hipMemcpyHostToDevice, s));
        BH(hipStreamSynchronize(s));
    }
    // Products run only on the columns that use them: the inner CG's on columns
    // in their cycle with an active CG, the Arnoldi step's on columns in their
    // cycle, the cycle-end residual's on columns that took a step this cycle.
    const ColGate gate_inner{B.in_cycle, B.cg_active}, gate_arnoldi{B.in_cycle, nullptr},
        gate_cycle_end{B.kcol, nullptr};
    auto products = [&](const void *Q, void *Yo, bool inner, ColGate gate, hipStream_t st) -> hipError_t {
        for (size_t c = 0; c < bp_in.size(); ++c)
            KRR_HIP(batched_product(inner ? bp_in[c] : bp_out[c], Q, Yo, inner ? 1 : 0, gate, st));
        return hipSuccess;
    };

    // the inner CG on fixed buffers (vin -> z32), recorded once as a graph
    const double tol2 = o.inner_tol * o.inner_tol;
    auto inner_seq = [&](hipStream_t st) -> hipError_t {
        hipLaunchKernelGGL(kb_cg_init, dim3(nb), dim3(BLOCK), 0, st, B, L.vin, L.z32, L.r32, L.p32);
        hipLaunchKernelGGL(kb_cg_init_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, tol2, o.inner_maxit);
        for (int it = 0; it < o.inner_maxit; ++it) {
            KRR_HIP(products(L.p32, L.Ap32, true, gate_inner, st));
            hipLaunchKernelGGL(kb_cg_alpha, dim3(nb), dim3(BLOCK), 0, st, B, L.p32, L.Ap32);
            hipLaunchKernelGGL(kb_cg_alpha_col, dim3(ccb), dim3(BLOCK), 0, st, B, C);
            hipLaunchKernelGGL(kb_cg_update, dim3(nb), dim3(BLOCK), 0, st, B, L.z32, L.r32, L.p32, L.Ap32);
            hipLaunchKernelGGL(kb_cg_update_col, dim3(ccb), dim3(BLOCK), 0, st, B, C, o.inner_maxit);
            hipLaunchKernelGGL(kb_cg_pupdate, dim3(nb), dim3(BLOCK), 0, st, B, L.r32, L.p32);
        }
        return hipGetLastError();
    };
    hipStream_t gs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    // KRR_NO_GRAPH=1 runs the same inner sequence eagerly (used to check that the
    // graph replays give bit-identical results)
    const char *nog = std::getenv("KRR_NO_GRAPH");
    bool use_graph = o.inner != KRR_INNER_NONE && !(nog && nog[0] == '1');
    auto cleanup = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (gs) (void)hipStreamDestroy(gs);
        if (ev_a) (void)hipEventDestroy(ev_a);
        if (ev_b) (void)hipEventDestroy(ev_b);
    };
    if (use_graph) {
        if (hipStreamCreateWithFlags(&gs, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&ev_a) != hipSuccess ||
            hipEventCreate(&ev_b) != hipSuccess) {
            cleanup();
            return KRR_EHIP;
        }
        profile_suspend(true);  // no timing events inside the recorded graph
        hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = inner_seq(gs);
        hipError_t e2 = hipStreamEndCapture(gs, &graph);
        profile_suspend(false);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            cleanup();
            return KRR_EHIP;
        }
    }
    auto run_inner = [&]() -> hipError_t {
        if (!use_graph) return inner_seq(s);
        KRR_HIP(hipEventRecord(ev_a, s));
        KRR_HIP(hipStreamWaitEvent(gs, ev_a, 0));
        KRR_HIP(hipGraphLaunch(gexec, gs));
        KRR_HIP(hipEventRecord(ev_b, gs));
        return hipStreamWaitEvent(s, ev_b, 0);
    };

    int outer = 0, cycles = 0, result = KRR_NOT_CONVERGED;
    int64_t mvp64 = 0, mvp_in = 0;
    int host[4];
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
    if (host[1] > 0) {
        cleanup();
        return KRR_ENONFINITE;
    }
    while (host[0] > 0 && outer < o.max_outer) {
        hipLaunchKernelGGL(kb_first_basis, dim3(nb), dim3(BLOCK), 0, s, B, L.r, L.V);
        for (int j = 0; j < m && outer < o.max_outer; ++j) {
            double *Vj = L.V + static_cast<int64_t>(j) * LL;
            double *Zj = L.Z + static_cast<int64_t>(j) * LL;
            if (o.inner == KRR_INNER_NONE) {
                hipLaunchKernelGGL(kb_copy, dim3(nb), dim3(BLOCK), 0, s, B, Vj, Zj);
            } else {
                hipLaunchKernelGGL(kb_copy, dim3(nb), dim3(BLOCK), 0, s, B, Vj, L.vin);
                BHC(run_inner());
                hipLaunchKernelGGL(kb_cast_z, dim3(nb), dim3(BLOCK), 0, s, B, L.z32, Zj);
                mvp_in += o.inner_maxit;
            }
            BHC(products(Zj, L.w, false, gate_arnoldi, s));
            ++mvp64;
            hipLaunchKernelGGL(kb_mgs_first, dim3(nb), dim3(BLOCK), 0, s, B, L.w, L.V);
            hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, 0, 0, m);
            for (int i = 0; i < j; ++i) {
                hipLaunchKernelGGL(kb_mgs_step, dim3(nb), dim3(BLOCK), 0, s, B, L.w, L.V + i * LL,
                                   L.V + (i + 1) * LL, i, m);
                hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, 1, i + 1, m);
            }
            hipLaunchKernelGGL(kb_mgs_last, dim3(nb), dim3(BLOCK), 0, s, B, L.w, Vj, j, m);
            hipLaunchKernelGGL(kb_mgs_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, 2, j + 1, m);
            // normalise before the Givens step decides whether the column leaves its cycle
            hipLaunchKernelGGL(kb_normalize, dim3(nb), dim3(BLOCK), 0, s, B, L.w, L.V + (j + 1) * LL, j, m);
            hipLaunchKernelGGL(kb_givens, dim3(cb), dim3(BLOCK), 0, s, B, C, j, m, o.tol);
            ++outer;
            BHC(read_summary());
            if (progress_every() && outer % progress_every() == 0)
                std::fprintf(stderr, "krr batched fgmres: outer %d cycle %d columns in their cycle %d of %d\n", outer,
                             cycles + 1, host[0], nprob * nrhs);
            if (host[0] == 0) break;
        }
        // x += Z y per column, then the true residual restarts the unconverged ones
        hipLaunchKernelGGL(kb_backsolve, dim3(cb), dim3(BLOCK), 0, s, B, C, m);
        hipLaunchKernelGGL(kb_update_x, dim3(nb), dim3(BLOCK), 0, s, B, L.Z, LL, m, L.x);
        ++cycles;
        BHC(products(L.x, L.w, false, gate_cycle_end, s));
        ++mvp64;
        hipLaunchKernelGGL(kb_residual, dim3(nb), dim3(BLOCK), 0, s, B, L.b, L.w, L.r);
        hipLaunchKernelGGL(kb_residual_col, dim3(ccb), dim3(BLOCK), 0, s, B, C, 1, m, o.tol);
        BHC(read_summary());
        if (host[1] > 0) {
            result = KRR_BREAKDOWN;
            break;
        }
    }
    if (result != KRR_BREAKDOWN) result = host[0] == 0 ? KRR_OK : KRR_NOT_CONVERGED;
    for (int k = 0; k < nprob; ++k) {
        const Sys &S = L.sys[k];
        const int64_t ld = ldy ? ldy[k] : probs[k].n;
        const int64_t tot = S.P.n_pad * nrhs;
        hipLaunchKernelGGL(kb_scatter, dim3((tot + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, S.P.perm, S.P.n_pad, nrhs,
                           L.x + S.base, W[k], ld);
    }
    std::vector<double> est(C), bn(C);
    BHC(hipMemcpyAsync(est.data(), B.est, sizeof(double) * C, hipMemcpyDeviceToHost, s));
    BHC(hipStreamSynchronize(s));
    cleanup();
    if (infos) {
        const double t = wall_ms() - t0;
        for (int k = 0; k < nprob; ++k)
            for (int r = 0; r < nrhs; ++r) {
                krr_info &I = infos[static_cast<size_t>(k) * nrhs + r];
                std::memset(&I, 0, sizeof(I));
                const double e = est[k * Rp + r];
                I.status = (e <= o.tol) ? KRR_OK : (result == KRR_BREAKDOWN ? KRR_BREAKDOWN : KRR_NOT_CONVERGED);
                I.outer_iters = outer;
                I.inner_iters = static_cast<int32_t>(mvp_in);
                I.cycles = cycles;
                I.mvp64 = mvp64;
                if (inner_prec == KRR_BF16) I.mvp16 = mvp_in;
                else I.mvp32 = mvp_in;
                I.relres_true = e;
                I.relres_est = e;
                I.t_total_ms = t;
            }
    }
    return result;
}

}  // namespace krr
