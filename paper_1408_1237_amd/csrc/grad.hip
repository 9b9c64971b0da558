// Adjoint pass for the gradient of a loss l(w), w = K^{-1} y, with respect to
// the points, log sigma and log gamma (hyperparameters by maximum likelihood,
// section 2.1).  With lambda = K^{-1} dl/dw, dl/dtheta = -lambda^T (dK/dtheta) w:
//   dl/dx_i   = (1/sigma^2) sum_j (lambda_i w_j + lambda_j w_i) K_hat_ij (x_i - x_j)
//   dl/dlogs  = -(1/sigma^2) sum_ij lambda_i w_j K_hat_ij ||x_i - x_j||^2
//   dl/dlogg  = -gamma lambda^T w.
// One pass over the pairs: per target row the kernel accumulates
//   Aw = sum_j K_hat_ij w_j D_ij,  Al = sum_j K_hat_ij lambda_j D_ij,
//   S  = sum_j K_hat_ij w_j ||D_ij||^2,
// with D_ij = x_i - x_j in scaled coordinates formed from tile anchors and
// offsets (t - o_j); the epilogue combines them with lambda_i, w_i in FP64.
// Sources arrive through scalar loads (wave-uniform addresses), as in the single
// product.  Precision: FP64 throughout (kernel values by exp2_f64), or FP32
// offsets, kernel values and sums.  At a solution w of an ill-conditioned system
// the row sums cancel heavily (|w| large with alternating signs), so the FP32
// gradient carries relative row errors far above FP32 rounding; FP64 costs about
// 1.8x the FP32 pass, small beside the solve that produces w.
#include "krylov.h"

namespace krr {

template <typename T>
struct GP;
template <>
struct GP<float> {
    static __device__ __forceinline__ float ex2(float a) { return __builtin_amdgcn_exp2f(a); }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};
template <>
struct GP<double> {
    static __device__ __forceinline__ double ex2(double a) { return exp2_f64(a); }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
};

struct GArgs {
    int64_t n, n_pad;
    int ntiles, nrowblocks, splits, tps;
    const double *anchor;
    const void *off;  // offsets in the pass's precision, SoA
    const void *ws;   // w in sorted order
    const void *ls;   // lambda in sorted order
    void *parts;      // [splits][n_pad][2D+1] (D+1 when lambda == w)
};

template <int D, bool SAME, typename T>
__global__ __launch_bounds__(BLOCK) void k_grad(GArgs a) {
    constexpr int NA = SAME ? D + 1 : 2 * D + 1;
    constexpr int U = D <= 4 ? 8 : D <= 8 ? 4 : 2;
    using G = GP<T>;
    const T *__restrict__ off = static_cast<const T *>(a.off);
    const T *__restrict__ wsrc = static_cast<const T *>(a.ws);
    const T *__restrict__ lsrc = static_cast<const T *>(a.ls);
    const int64_t n_pad = a.n_pad;
    const int bx = blockIdx.x % a.nrowblocks, by = blockIdx.x / a.nrowblocks;
    const int64_t i = static_cast<int64_t>(bx) * BLOCK + threadIdx.x;
    double aI[D];
    T oi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        aI[k] = a.anchor[static_cast<int64_t>(bx) * D + k];
        oi[k] = off[k * n_pad + i];
    }
    T Aw[D], Al[SAME ? 1 : D], S = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        Aw[k] = T(0);
        if (!SAME) Al[k] = T(0);
    }
    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    for (int J = J0; J < J1; ++J) {
        T t[D];
#pragma unroll
        for (int k = 0; k < D; ++k)
            t[k] = static_cast<T>((aI[k] - a.anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(oi[k]));
        const int64_t j0 = static_cast<int64_t>(J) * TILE;
        for (int jb = 0; jb < TILE; jb += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = j0 + jb + u;
                T dl[D];
                T r2 = T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    dl[k] = t[k] - off[k * n_pad + j];
                    r2 = G::fma(dl[k], dl[k], r2);
                }
                const T kv = G::ex2(-r2);
                const T kw = kv * wsrc[j];
                S = G::fma(kw, r2, S);
#pragma unroll
                for (int k = 0; k < D; ++k) Aw[k] = G::fma(kw, dl[k], Aw[k]);
                if (!SAME) {
                    const T kl = kv * lsrc[j];
#pragma unroll
                    for (int k = 0; k < D; ++k) Al[k] = G::fma(kl, dl[k], Al[k]);
                }
            }
        }
    }
    T *out = static_cast<T *>(a.parts) + (static_cast<int64_t>(by) * n_pad + i) * NA;
#pragma unroll
    for (int k = 0; k < D; ++k) out[k] = Aw[k];
    if (!SAME)
#pragma unroll
        for (int k = 0; k < D; ++k) out[D + k] = Al[k];
    out[NA - 1] = S;
}

// Sorted copies of lambda and w in the pass's precision (0 on the padding).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_grad_gather(const int32_t *__restrict__ perm, int64_t n_pad,
                                                       const double *__restrict__ lam, const double *__restrict__ w,
                                                       T *ls, T *ws) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (i >= n_pad) return;
    const int32_t p = perm[i];
    ls[i] = p >= 0 ? static_cast<T>(lam[p]) : T(0);
    ws[i] = p >= 0 ? static_cast<T>(w[p]) : T(0);
}

template <typename T>
__device__ __forceinline__ T gwave_sum(T v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o /= 2) v += __shfl_xor(v, o, WAVE);
    return v;
}

// gx[p_i, k] = (lambda_p Aw_k + w_p Al_k) / (sigma^2 c); sums lambda_p S_i and
// lambda_p w_p over rows (last block writes the two scalars).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_grad_finish(int64_t n, int64_t n_pad, int d, int dpad, int splits,
                                                       int same, const int32_t *__restrict__ perm,
                                                       const T *__restrict__ parts, const double *__restrict__ lam,
                                                       const double *__restrict__ w, double inv_s2c,
                                                       double inv_s2c2, double gamma, double *gx, double *g_ls,
                                                       double *g_lg, double *partials, unsigned *counter) {
    const int NA = same ? dpad + 1 : 2 * dpad + 1;
    double accS = 0.0, accG = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * BLOCK) {
        const int64_t p = perm[i];
        const double li = lam[p], wi = w[p];
        for (int k = 0; k < d; ++k) {
            double aw = 0.0, al = 0.0;
            for (int s = 0; s < splits; ++s) {
                const T *o = parts + (static_cast<int64_t>(s) * n_pad + i) * NA;
                aw += static_cast<double>(o[k]);
                al += static_cast<double>(o[same ? k : dpad + k]);
            }
            gx[p * d + k] = (li * aw + wi * al) * inv_s2c;
        }
        double S = 0.0;
        for (int s = 0; s < splits; ++s) S += static_cast<double>(parts[(static_cast<int64_t>(s) * n_pad + i) * NA + NA - 1]);
        accS += li * S;
        accG += li * wi;
    }
    // deterministic grid reduction of the two scalars (last block)
    __shared__ double sh[2][BLOCK / WAVE];
    __shared__ int is_last;
    accS = gwave_sum(accS);
    accG = gwave_sum(accG);
    if (threadIdx.x % WAVE == 0) {
        sh[0][threadIdx.x / WAVE] = accS;
        sh[1][threadIdx.x / WAVE] = accG;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int k = 0; k < BLOCK / WAVE; ++k) {
            a0 += sh[0][k];
            a1 += sh[1][k];
        }
        partials[blockIdx.x] = a0;
        partials[gridDim.x + blockIdx.x] = a1;
        __threadfence();
        is_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last || threadIdx.x != 0) return;
    __threadfence();
    double s0 = 0.0, s1 = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) {
        s0 += __hip_atomic_load(&partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s1 += __hip_atomic_load(&partials[gridDim.x + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    *g_ls = -s0 * inv_s2c2;
    *g_lg = -gamma * s1;
    *counter = 0u;
}

__global__ void k_zero_u32(unsigned *p) {
    if (threadIdx.x == 0) *p = 0u;
}

// ---------------------------------------------------------------- host

static int grad_splits(const Prepared &P) {
    int s = (4096 + P.ntiles - 1) / P.ntiles;
    int mx = P.ntiles / 2 > 1 ? P.ntiles / 2 : 1;
    if (mx > 32) mx = 32;
    if (s > mx) s = mx;
    return s < 1 ? 1 : s;
}

size_t grad_scratch_bytes(const Prepared &P) {
    const int mx = (P.ntiles / 2 > 1 ? (P.ntiles / 2 < 32 ? P.ntiles / 2 : 32) : 1);
    return align_up(static_cast<size_t>(mx) * P.n_pad * (2 * P.dpad + 1) * 8, 256) +
           2 * align_up(static_cast<size_t>(P.n_pad) * 8, 256) + align_up(2 * VEC_BLOCKS * 8, 256) + 256;
}

template <int D, typename T>
static hipError_t launch_grad(const GArgs &a, bool same, hipStream_t s) {
    if (same)
        hipLaunchKernelGGL((k_grad<D, true, T>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((k_grad<D, false, T>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t grad_pass(const Prepared &P, double sigma, double gamma, const double *lam, const double *w,
                            double *gx, double *g_ls, double *g_lg, void *scratch, hipStream_t s) {
    const bool same = (lam == w);
    const int mx = (P.ntiles / 2 > 1 ? (P.ntiles / 2 < 32 ? P.ntiles / 2 : 32) : 1);
    Carver cv(scratch);
    GArgs a;
    T *parts = cv.take<T>(static_cast<size_t>(mx) * P.n_pad * (2 * P.dpad + 1));
    T *ls = cv.take<T>(P.n_pad);
    T *wsv = cv.take<T>(P.n_pad);
    double *partials = cv.take<double>(2 * VEC_BLOCKS);
    unsigned *counter = cv.take<unsigned>(1);
    const int splits_req = grad_splits(P);
    a.n = P.n;
    a.n_pad = P.n_pad;
    a.ntiles = P.ntiles;
    a.nrowblocks = P.ntiles;
    a.tps = (P.ntiles + splits_req - 1) / splits_req;
    a.splits = (P.ntiles + a.tps - 1) / a.tps;
    a.anchor = P.anchor;
    a.off = sizeof(T) == 8 ? static_cast<const void *>(P.off64) : static_cast<const void *>(P.off32);
    a.ws = wsv;
    a.ls = ls;
    a.parts = parts;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counter);
    hipLaunchKernelGGL(k_grad_gather<T>, dim3((P.n_pad + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, P.perm, P.n_pad, lam,
                       w, ls, wsv);
    KRR_HIP(hipGetLastError());
    hipError_t e;
    switch (P.dpad) {
        case 1: e = launch_grad<1, T>(a, same, s); break;
        case 2: e = launch_grad<2, T>(a, same, s); break;
        case 3: e = launch_grad<3, T>(a, same, s); break;
        case 4: e = launch_grad<4, T>(a, same, s); break;
        case 6: e = launch_grad<6, T>(a, same, s); break;
        case 8: e = launch_grad<8, T>(a, same, s); break;
        case 12: e = launch_grad<12, T>(a, same, s); break;
        case 16: e = launch_grad<16, T>(a, same, s); break;
        case 24: e = launch_grad<24, T>(a, same, s); break;
        case 32: e = launch_grad<32, T>(a, same, s); break;
        case 48: e = launch_grad<48, T>(a, same, s); break;
        case 64: e = launch_grad<64, T>(a, same, s); break;
        default: e = hipErrorInvalidValue;
    }
    KRR_HIP(e);
    const double c = P.scale;
    const double s2 = sigma * sigma;
    hipLaunchKernelGGL(k_grad_finish<T>, dim3(vec_blocks(P.n_pad)), dim3(BLOCK), 0, s, P.n, P.n_pad, P.d, P.dpad,
                       a.splits, same ? 1 : 0, P.perm, parts, lam, w, 1.0 / (s2 * c), 1.0 / (s2 * c * c), gamma,
                       gx, g_ls, g_lg, partials, counter);
    return hipGetLastError();
}

hipError_t kmvp_grad_run(const Prepared &P, int prec, double sigma, double gamma, const double *lam,
                         const double *w, double *gx, double *g_ls, double *g_lg, void *scratch, hipStream_t s) {
    if (prec == KRR_FP64) return grad_pass<double>(P, sigma, gamma, lam, w, gx, g_ls, g_lg, scratch, s);
    return grad_pass<float>(P, sigma, gamma, lam, w, gx, g_ls, g_lg, scratch, s);
}

}  // namespace krr
