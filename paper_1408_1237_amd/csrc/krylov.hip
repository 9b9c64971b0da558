// Krylov vector kernels: CG steps, Gram-Schmidt, Givens least squares.
//
// Every reduction is deterministic: each block reduces its grid-stride slice
// with wavefront shuffles and LDS, writes one partial, and the last block to
// arrive (found with a device-scope atomic counter) adds the partials in block
// order and applies the scalar epilogue (CG step lengths, Hessenberg entries,
// convergence flags).  Solver scalars stay in device memory, so no kernel waits
// for the host.  All vectors are sorted, zero-padded, of length n_pad.
#include "krylov.h"

namespace krr {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off /= 2) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Sum over the block; the result is valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v) {
    __shared__ T sh[BLOCK / WAVE];
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x % WAVE) == 0) sh[threadIdx.x / WAVE] = v;
    __syncthreads();
    T r = T(0);
    if (threadIdx.x == 0)
        for (int k = 0; k < BLOCK / WAVE; ++k) r += sh[k];
    return r;
}

// Grid-wide sum of NV values by the last-block pattern.  Returns true in the
// last block only; there v[] holds the totals in thread 0.
template <typename T, int NV>
__device__ bool grid_reduce(T (&v)[NV], T *partials, unsigned *counter) {
    __shared__ int is_last;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = block_sum(v[k]);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[k * gridDim.x + blockIdx.x] = v[k];
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        T s = T(0);
        for (unsigned b = threadIdx.x; b < gridDim.x; b += BLOCK)
            s += __hip_atomic_load(&partials[k * gridDim.x + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v[k] = block_sum(s);
    }
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x; i < (n); i += static_cast<int64_t>(gridDim.x) * BLOCK)

// ------------------------------------------------------------------ CG

// x = 0, r = p = rhs, rr = rr0 = r.r; stop threshold tol2 * rr0.
template <typename T, typename TV>
__global__ __launch_bounds__(BLOCK) void k_cg_init(int64_t n_pad, const TV *__restrict__ rhs, T *x, T *r, T *p,
                                                   uint16_t *p16, CgScalars<T> *S, double tol2, int maxit,
                                                   T *partials, unsigned *counter) {
    T acc[1] = {T(0)};
    GRID_STRIDE(i, n_pad) {
        const T v = static_cast<T>(rhs[i]);
        x[i] = T(0);
        r[i] = v;
        p[i] = v;
        if (p16) p16[i] = f32_to_bf16_rne(static_cast<float>(v));
        acc[0] += v * v;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        const T rr = acc[0];
        S->rr = rr;
        S->rr0 = rr;
        S->thresh = static_cast<T>(tol2 * static_cast<double>(rr));
        S->alpha = S->beta = S->pAp = T(0);
        S->iters = 0;
        S->maxit = maxit;
        S->status = isfinite(static_cast<double>(rr)) ? 0 : KRR_ENONFINITE;
        S->candidate = (rr == T(0)) ? 1 : 0;
        S->active = (rr > T(0) && maxit > 0 && S->status == 0) ? 1 : 0;
    }
}

// pAp = p . Ap, alpha = rr / pAp (breakdown when pAp <= 0 or not finite).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cg_alpha(int64_t n_pad, const T *__restrict__ p, const T *__restrict__ Ap,
                                                    CgScalars<T> *S, T *partials, unsigned *counter) {
    if (S->active == 0) return;
    T acc[1] = {T(0)};
    GRID_STRIDE(i, n_pad) acc[0] += p[i] * Ap[i];
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        const T pAp = acc[0];
        if (!(pAp > T(0)) || !isfinite(static_cast<double>(pAp))) {
            S->status = KRR_BREAKDOWN;
            S->active = 0;
        } else {
            S->pAp = pAp;
            S->alpha = S->rr / pAp;
        }
    }
}

// x += alpha p, r -= alpha Ap, rr' = r.r, beta = rr'/rr; stop tests.  With a
// history array, iteration k stores (alpha_k, beta_k) at hist[2k], hist[2k+1]
// while k < hist_cap (the coefficients of the Lanczos tridiagonal).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cg_update(int64_t n_pad, T *x, T *r, const T *__restrict__ p,
                                                     const T *__restrict__ Ap, CgScalars<T> *S, T *partials,
                                                     unsigned *counter, double *hist, int hist_cap) {
    if (S->active == 0) return;
    const T a = S->alpha;
    T acc[1] = {T(0)};
    GRID_STRIDE(i, n_pad) {
        x[i] += a * p[i];
        const T ri = r[i] - a * Ap[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        const T rr = acc[0];
        S->beta = rr / S->rr;
        S->rr = rr;
        if (hist != nullptr && S->iters < hist_cap) {
            hist[2 * S->iters] = static_cast<double>(S->alpha);
            hist[2 * S->iters + 1] = static_cast<double>(S->beta);
        }
        S->iters += 1;
        if (!isfinite(static_cast<double>(rr))) {
            S->status = KRR_BREAKDOWN;
            S->active = 0;
        } else if (rr <= S->thresh) {
            S->candidate = 1;
            S->active = 0;
        } else if (S->iters >= S->maxit) {
            S->active = 0;
        }
    }
}

// p = r + beta p (and its bf16 copy for the bf16 product).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cg_pupdate(int64_t n_pad, const T *__restrict__ r, T *p, uint16_t *p16,
                                                      const CgScalars<T> *S) {
    if (S->active == 0) return;
    const T b = S->beta;
    GRID_STRIDE(i, n_pad) {
        const T v = r[i] + b * p[i];
        p[i] = v;
        if (p16) p16[i] = f32_to_bf16_rne(static_cast<float>(v));
    }
}

// Restart of the plain solver from its true residual: r = p = b - Kx,
// rr = r.r; iterate again when rr is above the threshold.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cg_restart(int64_t n_pad, const T *__restrict__ b, const T *__restrict__ Kx,
                                                      T *r, T *p, CgScalars<T> *S, T *partials, unsigned *counter) {
    T acc[1] = {T(0)};
    GRID_STRIDE(i, n_pad) {
        const T v = b[i] - Kx[i];
        r[i] = v;
        p[i] = v;
        acc[0] += v * v;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        const T rr = acc[0];
        S->rr = rr;
        S->candidate = (rr <= S->thresh) ? 1 : 0;
        S->active = (S->candidate == 0 && S->iters < S->maxit && isfinite(static_cast<double>(rr))) ? 1 : 0;
    }
}

// ------------------------------------------------------------------ FGMRES

// r = b - Kx (Kx may be null: x = 0; r may alias Kx); beta = ||r||,
// bnorm = ||b||, g = beta e1, est = beta / bnorm.
__global__ __launch_bounds__(BLOCK) void k_fg_residual(int64_t n_pad, const double *__restrict__ b,
                                                       const double *Kx, double *r, FgmresScalars *F,
                                                       double *g, double *partials, unsigned *counter) {
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, n_pad) {
        const double bi = b[i];
        const double v = Kx ? bi - Kx[i] : bi;
        r[i] = v;
        acc[0] += v * v;
        acc[1] += bi * bi;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        const double beta = sqrt(acc[0]), bn = sqrt(acc[1]);
        F->beta = beta;
        F->bnorm = bn;
        F->est = bn > 0.0 ? beta / bn : 0.0;
        F->breakdown = 0;
        F->nonfinite = (isfinite(beta) && isfinite(bn)) ? 0 : 1;
        g[0] = beta;
    }
}

// v = r / beta
__global__ __launch_bounds__(BLOCK) void k_fg_first_basis(int64_t n_pad, const double *__restrict__ r, double *v,
                                                          const FgmresScalars *F) {
    const double inv = 1.0 / F->beta;
    GRID_STRIDE(i, n_pad) v[i] = r[i] * inv;
}

__global__ __launch_bounds__(BLOCK) void k_cast_f2d(int64_t n_pad, const float *__restrict__ z, double *Zj) {
    GRID_STRIDE(i, n_pad) Zj[i] = static_cast<double>(z[i]);
}

__global__ __launch_bounds__(BLOCK) void k_copy_d(int64_t n_pad, const double *__restrict__ a, double *b) {
    GRID_STRIDE(i, n_pad) b[i] = a[i];
}

// MGS, first projection: h_0j = w . v_0, and ||w|| before orthogonalisation.
__global__ __launch_bounds__(BLOCK) void k_mgs_first(int64_t n_pad, const double *__restrict__ w,
                                                     const double *__restrict__ v0, double *hcol, FgmresScalars *F,
                                                     double *partials, unsigned *counter) {
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, n_pad) {
        const double wi = w[i];
        acc[0] += wi * v0[i];
        acc[1] += wi * wi;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        hcol[0] = acc[0];
        F->wnorm0 = sqrt(acc[1]);
    }
}

// MGS step: w -= h_ij v_i, then h_{i+1,j} = w . v_{i+1}.
__global__ __launch_bounds__(BLOCK) void k_mgs_step(int64_t n_pad, double *w, const double *__restrict__ vi,
                                                    const double *__restrict__ vnext, double *hcol, int i_,
                                                    double *partials, unsigned *counter) {
    const double h = hcol[i_];
    double acc[1] = {0.0};
    GRID_STRIDE(i, n_pad) {
        const double wi = w[i] - h * vi[i];
        w[i] = wi;
        acc[0] += wi * vnext[i];
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) hcol[i_ + 1] = acc[0];
}

// MGS last: w -= h_jj v_j, h_{j+1,j} = ||w||.
__global__ __launch_bounds__(BLOCK) void k_mgs_last(int64_t n_pad, double *w, const double *__restrict__ vj,
                                                    double *hcol, int j, double *partials, unsigned *counter) {
    const double h = hcol[j];
    double acc[1] = {0.0};
    GRID_STRIDE(i, n_pad) {
        const double wi = w[i] - h * vj[i];
        w[i] = wi;
        acc[0] += wi * wi;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) hcol[j + 1] = sqrt(acc[0]);
}

// Classical Gram-Schmidt projection for one pass: hpass = V[:, 0..j]^T w, and
// hcol[0..j] = hpass (hacc = 0) or hcol[0..j] += hpass (hacc = 1).  Each block
// forms partials of all j+1 dot products.
__global__ __launch_bounds__(BLOCK) void k_cgs_dots(int64_t n_pad, const double *__restrict__ w,
                                                    const double *__restrict__ V, int j, double *hpass,
                                                    double *hcol, int hacc, double *partials, unsigned *counter) {
    __shared__ int is_last;
    for (int c = 0; c <= j; ++c) {
        double s = 0.0;
        const double *vc = V + static_cast<int64_t>(c) * n_pad;
        GRID_STRIDE(i, n_pad) s += w[i] * vc[i];
        s = block_sum(s);
        if (threadIdx.x == 0) partials[c * gridDim.x + blockIdx.x] = s;
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    for (int c = 0; c <= j; ++c) {
        double s = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += BLOCK)
            s += __hip_atomic_load(&partials[c * gridDim.x + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = block_sum(s);
        if (threadIdx.x == 0) {
            hpass[c] = s;
            hcol[c] = hacc ? hcol[c] + s : s;
        }
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// w -= V[:, 0..j] h (hcur: the pass's own coefficients); optional ||w||^2 into hcol[j+1].
__global__ __launch_bounds__(BLOCK) void k_cgs_sub(int64_t n_pad, double *w, const double *__restrict__ V, int j,
                                                   const double *__restrict__ hcur, double *hcol, int want_norm,
                                                   double *partials, unsigned *counter) {
    double acc[1] = {0.0};
    GRID_STRIDE(i, n_pad) {
        double wi = w[i];
        for (int c = 0; c <= j; ++c) wi -= hcur[c] * V[static_cast<int64_t>(c) * n_pad + i];
        w[i] = wi;
        acc[0] += wi * wi;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0 && want_norm) hcol[j + 1] = sqrt(acc[0]);
}

// Least squares by Givens rotations: rotate column j of H_bar with the
// previous rotations, form rotation j, update g; residual estimate
// |g_{j+1}| / ||b||; happy breakdown when h_{j+1,j} <= 1e-14 ||K z_j||.
// H holds the rotated columns, column-major with leading dimension m+1.
__global__ void k_givens(int j, int m, const double *hcol, double *H, double *cs, double *sn, double *g,
                         FgmresScalars *F) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double *col = H + static_cast<int64_t>(j) * (m + 1);
    for (int i = 0; i <= j + 1; ++i) col[i] = hcol[i];
    for (int i = 0; i < j; ++i) {
        const double a = col[i], c = col[i + 1];
        col[i] = cs[i] * a + sn[i] * c;
        col[i + 1] = -sn[i] * a + cs[i] * c;
    }
    const double a = col[j], c = col[j + 1];
    const double rho = sqrt(a * a + c * c);
    cs[j] = a / rho;
    sn[j] = c / rho;
    col[j] = rho;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    F->breakdown = (hcol[j + 1] > 1e-14 * F->wnorm0) ? 0 : 1;
    F->est = fabs(g[j + 1]) / F->bnorm;
    if (!isfinite(F->est)) F->nonfinite = 1;
}

// v_{j+1} = w / h_{j+1,j} (not after a breakdown)
__global__ __launch_bounds__(BLOCK) void k_fg_normalize(int64_t n_pad, const double *__restrict__ w, double *vnext,
                                                        const double *hcol, int j, const FgmresScalars *F) {
    if (F->breakdown) return;
    const double inv = 1.0 / hcol[j + 1];
    GRID_STRIDE(i, n_pad) vnext[i] = w[i] * inv;
}

// y = R^{-1} g[0..k-1] (R: the rotated H, upper triangular)
__global__ void k_fg_backsolve(int k, int m, const double *H, const double *g, double *y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int t = i + 1; t < k; ++t) s -= H[static_cast<int64_t>(t) * (m + 1) + i] * y[t];
        y[i] = s / H[static_cast<int64_t>(i) * (m + 1) + i];
    }
}

// x += Z[:, 0..k-1] y
__global__ __launch_bounds__(BLOCK) void k_fg_update_x(int64_t n_pad, int k, const double *__restrict__ Z,
                                                       const double *__restrict__ y, double *x) {
    GRID_STRIDE(i, n_pad) {
        double s = x[i];
        for (int c = 0; c < k; ++c) s += Z[static_cast<int64_t>(c) * n_pad + i] * y[c];
        x[i] = s;
    }
}

__global__ void k_fill_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_fill_d(double *p, int64_t n, double v) {
    GRID_STRIDE(i, n) p[i] = v;
}

__global__ void k_fill_bytes(unsigned char *p, int64_t n) {
    GRID_STRIDE(i, n) p[i] = 0;
}

// ------------------------------------------------------------------ host launchers

int vec_blocks(int64_t n_pad) {
    const int64_t b = (n_pad + BLOCK - 1) / BLOCK;
    return static_cast<int>(b < VEC_BLOCKS ? b : VEC_BLOCKS);
}

#define LAUNCH(kern, grid, ...) hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), 0, s, __VA_ARGS__)

hipError_t red_init(const Red &R, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, R.counters, Red::NCOUNTERS);
    return hipGetLastError();
}

template <typename T, typename TV>
hipError_t cg_init(const CgVecs<T> &c, const TV *rhs, double tol, int maxit, const Red &R, hipStream_t s) {
    LAUNCH((k_cg_init<T, TV>), vec_blocks(c.n_pad), c.n_pad, rhs, c.x, c.r, c.p, c.p16, c.S, tol * tol, maxit,
           reinterpret_cast<T *>(R.partials), R.counters + 0);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_step(const Prepared &P, int prec, double shift, const CgVecs<T> &c, const KmvpScratch &sc,
                   const Red &R, hipStream_t s) {
    const void *qin = (prec == KRR_BF16) ? static_cast<const void *>(c.p16) : static_cast<const void *>(c.p);
    KRR_HIP(kmvp_sorted(P, prec, shift, qin, c.Ap, sc, &c.S->active, s));
    const int nb = vec_blocks(c.n_pad);
    T *part = reinterpret_cast<T *>(R.partials);
    LAUNCH(k_cg_alpha<T>, nb, c.n_pad, c.p, c.Ap, c.S, part, R.counters + 1);
    LAUNCH(k_cg_update<T>, nb, c.n_pad, c.x, c.r, c.p, c.Ap, c.S, part, R.counters + 2, c.hist, c.hist_cap);
    LAUNCH(k_cg_pupdate<T>, nb, c.n_pad, c.r, c.p, c.p16, c.S);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_restart(const CgVecs<T> &c, const T *b, const T *Kx, const Red &R, hipStream_t s) {
    LAUNCH(k_cg_restart<T>, vec_blocks(c.n_pad), c.n_pad, b, Kx, c.r, c.p, c.S, reinterpret_cast<T *>(R.partials),
           R.counters + 3);
    return hipGetLastError();
}

template hipError_t cg_init<float, double>(const CgVecs<float> &, const double *, double, int, const Red &,
                                           hipStream_t);
template hipError_t cg_init<float, float>(const CgVecs<float> &, const float *, double, int, const Red &,
                                          hipStream_t);
template hipError_t cg_init<double, double>(const CgVecs<double> &, const double *, double, int, const Red &,
                                            hipStream_t);
template hipError_t cg_step<float>(const Prepared &, int, double, const CgVecs<float> &, const KmvpScratch &,
                                   const Red &, hipStream_t);
template hipError_t cg_step<double>(const Prepared &, int, double, const CgVecs<double> &, const KmvpScratch &,
                                    const Red &, hipStream_t);
template hipError_t cg_restart<double>(const CgVecs<double> &, const double *, const double *, const Red &,
                                       hipStream_t);

hipError_t fg_residual(int64_t n_pad, const double *b, const double *Kx, double *r, FgmresScalars *F, double *g,
                       const Red &R, hipStream_t s) {
    LAUNCH(k_fg_residual, vec_blocks(n_pad), n_pad, b, Kx, r, F, g, R.partials, R.counters + 4);
    return hipGetLastError();
}

hipError_t fg_first_basis(int64_t n_pad, const double *r, double *v, const FgmresScalars *F, hipStream_t s) {
    LAUNCH(k_fg_first_basis, vec_blocks(n_pad), n_pad, r, v, F);
    return hipGetLastError();
}

hipError_t cast_f2d(int64_t n_pad, const float *z, double *Zj, hipStream_t s) {
    LAUNCH(k_cast_f2d, vec_blocks(n_pad), n_pad, z, Zj);
    return hipGetLastError();
}

hipError_t copy_d(int64_t n_pad, const double *a, double *b, hipStream_t s) {
    LAUNCH(k_copy_d, vec_blocks(n_pad), n_pad, a, b);
    return hipGetLastError();
}

hipError_t fill_d(double *p, int64_t n, double v, hipStream_t s) {
    LAUNCH(k_fill_d, vec_blocks(n), p, n, v);
    return hipGetLastError();
}

hipError_t zero_bytes(void *p, int64_t n, hipStream_t s) {
    LAUNCH(k_fill_bytes, vec_blocks(n), static_cast<unsigned char *>(p), n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ flexible CG

// beta_k = (z . q_k) / (d_k . q_k) for the stored directions; 0 for the slot the
// new direction is about to replace.
__global__ void k_fcg_beta(int nslots, int cur, const double *hcol, const double *dq, double *beta) {
    for (int k = threadIdx.x; k < nslots; k += blockDim.x) beta[k] = (k == cur) ? 0.0 : hcol[k] / dq[k];
}

// dq[cur] = d . q, alpha = (d . r) / (d . q); breakdown when d . q <= 0.
__global__ __launch_bounds__(BLOCK) void k_fcg_alpha(int64_t n_pad, const double *__restrict__ d,
                                                     const double *__restrict__ q, const double *__restrict__ r,
                                                     double *dq, int cur, double *alpha, FgmresScalars *F,
                                                     double *partials, unsigned *counter) {
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(i, n_pad) {
        acc[0] += d[i] * q[i];
        acc[1] += d[i] * r[i];
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        dq[cur] = acc[0];
        *alpha = acc[1] / acc[0];
        if (!(acc[0] > 0.0) || !isfinite(acc[0]) || !isfinite(acc[1])) F->breakdown = 1;
    }
}

// x += alpha d, r -= alpha q; est = ||r|| / ||b||.
__global__ __launch_bounds__(BLOCK) void k_fcg_update(int64_t n_pad, double *x, double *r,
                                                      const double *__restrict__ d, const double *__restrict__ q,
                                                      const double *alpha, FgmresScalars *F, double *partials,
                                                      unsigned *counter) {
    if (F->breakdown) return;  // uniform: set by the previous kernel
    const double a = *alpha;
    double acc[1] = {0.0};
    GRID_STRIDE(i, n_pad) {
        x[i] += a * d[i];
        const double ri = r[i] - a * q[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    if (grid_reduce(acc, partials, counter) && threadIdx.x == 0) {
        F->est = sqrt(acc[0]) / F->bnorm;
        if (!isfinite(F->est)) F->nonfinite = 1;
    }
}

hipError_t fg_orthogonalize(int gs, int64_t n_pad, int j, double *w, const double *V, double *hcol, double *hscratch,
                            FgmresScalars *F, const Red &R, hipStream_t s) {
    const int nb = vec_blocks(n_pad);
    if (gs == KRR_GS_MGS) {
        LAUNCH(k_mgs_first, nb, n_pad, w, V, hcol, F, R.partials, R.counters + 5);
        for (int i = 0; i < j; ++i)
            LAUNCH(k_mgs_step, nb, n_pad, w, V + static_cast<int64_t>(i) * n_pad,
                   V + static_cast<int64_t>(i + 1) * n_pad, hcol, i, R.partials, R.counters + 6);
        LAUNCH(k_mgs_last, nb, n_pad, w, V + static_cast<int64_t>(j) * n_pad, hcol, j, R.partials, R.counters + 7);
    } else {
        // two passes of classical Gram-Schmidt; ||w|| before projection first
        LAUNCH(k_mgs_first, nb, n_pad, w, V, hcol, F, R.partials, R.counters + 5);
        for (int pass = 0; pass < 2; ++pass) {
            LAUNCH(k_cgs_dots, nb, n_pad, w, V, j, hscratch, hcol, pass, R.partials, R.counters + 8);
            LAUNCH(k_cgs_sub, nb, n_pad, w, V, j, hscratch, hcol, pass, R.partials, R.counters + 9);
        }
    }
    return hipGetLastError();
}

hipError_t fg_givens(int j, int m, const double *hcol, double *H, double *cs, double *sn, double *g,
                     FgmresScalars *F, hipStream_t s) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, j, m, hcol, H, cs, sn, g, F);
    return hipGetLastError();
}

hipError_t fg_normalize(int64_t n_pad, const double *w, double *vnext, const double *hcol, int j,
                        const FgmresScalars *F, hipStream_t s) {
    LAUNCH(k_fg_normalize, vec_blocks(n_pad), n_pad, w, vnext, hcol, j, F);
    return hipGetLastError();
}

hipError_t fg_update_x(int64_t n_pad, int k, int m, const double *H, const double *g, double *y, const double *Z,
                       double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_fg_backsolve, dim3(1), dim3(64), 0, s, k, m, H, g, y);
    LAUNCH(k_fg_update_x, vec_blocks(n_pad), n_pad, k, Z, y, x);
    return hipGetLastError();
}

hipError_t fcg_direction(int64_t n_pad, int nslots, int cur, double *z, const double *D, const double *Q,
                         double *hcol, double *hpass, double *dq_beta_scratch, const double *dq, const Red &R,
                         hipStream_t s) {
    // z <- z - D beta with beta_k = (z . q_k) / (d_k . q_k)
    const int nb = vec_blocks(n_pad);
    if (nslots <= 0) return hipSuccess;
    LAUNCH(k_cgs_dots, nb, n_pad, z, Q, nslots - 1, hpass, hcol, 0, R.partials, R.counters + 10);
    hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(BLOCK), 0, s, nslots, cur, hcol, dq, dq_beta_scratch);
    LAUNCH(k_cgs_sub, nb, n_pad, z, D, nslots - 1, dq_beta_scratch, hcol, 0, R.partials, R.counters + 11);
    return hipGetLastError();
}

hipError_t fcg_step(int64_t n_pad, const double *d, const double *q, double *x, double *r, double *dq, int cur,
                    double *alpha, FgmresScalars *F, const Red &R, hipStream_t s) {
    const int nb = vec_blocks(n_pad);
    LAUNCH(k_fcg_alpha, nb, n_pad, d, q, r, dq, cur, alpha, F, R.partials, R.counters + 12);
    LAUNCH(k_fcg_update, nb, n_pad, x, r, d, q, alpha, F, R.partials, R.counters + 13);
    return hipGetLastError();
}

}  // namespace krr
