// On-the-fly Gaussian kernel products y = K_hat q + shift q (the weighted kernel
// summation of section 1 / section 3.1, with the shift of eq. RegKernel or of
// the preconditioner M = K_hat + delta I of section 5), single right-hand side.
//
// Work decomposition: one lane per target row; a block of 256 lanes covers one
// row tile.  The source columns are split into `splits` contiguous ranges of
// whole tiles (one block per (row tile, column range)); with splits > 1 a
// second kernel adds the partial sums in a fixed order (deterministic).  The
// source data of a column tile (offsets, weights, q) is read at wave-uniform
// addresses, so it arrives through scalar loads into SGPRs and feeds the VALU
// directly: no LDS staging and no barriers.  Per pair the folded form costs d
// fused multiply-adds, one exp2 and one accumulate (layout in krr_internal.h).
#include "krr_internal.h"

namespace krr {

// 2^a in FP64 for a <= 1023.  a = n + f with n = rint(a) and |f| <= 1/2 (the
// subtraction is exact), 2^f = e^(f ln 2) from its Taylor series to degree 12
// (truncation error below 2.4e-16 for |f ln 2| <= 0.347), scaled by 2^n.
// Arguments below -1100 are clamped (the result then underflows to 0).
__device__ __forceinline__ double exp2_f64(double a) {
    a = fmax(a, -1100.0);
    const double n = __builtin_rint(a);
    const double f = a - n;
    double p = 2.5678435993488206e-11;
    p = __builtin_fma(p, f, 4.4455382718708116e-10);
    p = __builtin_fma(p, f, 7.054911620801123e-09);
    p = __builtin_fma(p, f, 1.01780860092397e-07);
    p = __builtin_fma(p, f, 1.321548679014431e-06);
    p = __builtin_fma(p, f, 1.5252733804059841e-05);
    p = __builtin_fma(p, f, 0.0001540353039338161);
    p = __builtin_fma(p, f, 0.0013333558146428443);
    p = __builtin_fma(p, f, 0.009618129107628477);
    p = __builtin_fma(p, f, 0.05550410866482158);
    p = __builtin_fma(p, f, 0.24022650695910072);
    p = __builtin_fma(p, f, 0.6931471805599453);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_amdgcn_ldexp(p, static_cast<int>(n));
}

// Block index remap: consecutive hardware block ids are dealt round-robin to
// the 8 XCDs; give each XCD a contiguous range of logical blocks so that the
// blocks sharing a column range (and its source data in L2) run on one XCD.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int tall = nb / 8, extra = nb % 8;
    const int xcd = b % 8, local = b / 8;
    return xcd < extra ? xcd * (tall + 1) + local : extra * (tall + 1) + (xcd - extra) * tall + local;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int PREC>
struct Prec;
template <>
struct Prec<KRR_FP64> {
    using T = double;
    using Off = double;
    using Q = double;
    static constexpr double wide = WIDE_R2_FP64;
    static __device__ __forceinline__ T off(Off v) { return v; }
    static __device__ __forceinline__ T q(Q v) { return v; }
    static __device__ __forceinline__ T ex2(T a) { return exp2_f64(a); }
};
template <>
struct Prec<KRR_FP32> {
    using T = float;
    using Off = float;
    using Q = float;
    static constexpr double wide = WIDE_R2_FP32;
    static __device__ __forceinline__ T off(Off v) { return v; }
    static __device__ __forceinline__ T q(Q v) { return v; }
    static __device__ __forceinline__ T ex2(T a) { return __builtin_amdgcn_exp2f(a); }
};
template <>
struct Prec<KRR_BF16> {
    using T = float;
    using Off = uint16_t;
    using Q = uint16_t;
    static constexpr double wide = WIDE_R2_FP32;
    static __device__ __forceinline__ T off(Off v) { return bf16_to_f32(v); }
    static __device__ __forceinline__ T q(Q v) { return bf16_to_f32(v); }
    static __device__ __forceinline__ T ex2(T a) { return __builtin_amdgcn_exp2f(a); }
};

// Columns per unrolled step: keeps (D + 2) * U source words in SGPRs <= 64.
template <int D, int PREC>
constexpr int unroll_cols() {
    constexpr int words = (PREC == KRR_FP64 ? 2 : 1) * (D + 2);
    constexpr int u = 64 / words;
    return u >= 16 ? 16 : u >= 8 ? 8 : u >= 4 ? 4 : u >= 2 ? 2 : 1;
}

struct KArgs {
    int64_t n, n_pad;
    int ntiles, nrowblocks, splits, tps;
    const double *anchor;
    const double *tile_r2;
    const double *tile_nj;
    const void *off;
    const void *w;
    const void *q;
    void *out;
    double shift;
    const int *active;
};

template <int D, int PREC>
__global__ __launch_bounds__(BLOCK) void k_kmvp(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    using Off = typename P::Off;
    using Q = typename P::Q;
    constexpr int U = unroll_cols<D, PREC>();
    const Off *__restrict__ off = static_cast<const Off *>(a.off);
    const T *__restrict__ w = static_cast<const T *>(a.w);
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const double *__restrict__ anchor = a.anchor;
    const int64_t n_pad = a.n_pad;

    const int lb = xcd_remap(blockIdx.x, a.nrowblocks * a.splits);
    const int bx = lb % a.nrowblocks, by = lb / a.nrowblocks;
    const int64_t i = static_cast<int64_t>(bx) * BLOCK + threadIdx.x;

    double aI[D];
    T oi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        aI[k] = anchor[static_cast<int64_t>(bx) * D + k];
        oi[k] = P::off(off[k * n_pad + i]);
    }
    T acc = T(0);
    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    for (int J = J0; J < J1; ++J) {
        const double r2 = a.tile_r2[J];
        const double nj = a.tile_nj[J];
        T t[D];
        double tt = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double td = (aI[k] - anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(oi[k]);
            t[k] = static_cast<T>(td);
            const double tk = static_cast<double>(t[k]);
            tt = __builtin_fma(tk, tk, tt);
        }
        const int64_t j0 = static_cast<int64_t>(J) * TILE;
        if (r2 <= P::wide) {
            T Tk[D];
#pragma unroll
            for (int k = 0; k < D; ++k) Tk[k] = t[k] + t[k];
            const T c = static_cast<T>(-tt - nj);
            for (int jb = 0; jb < TILE; jb += U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t j = j0 + jb + u;
                    const T qq = P::q(q[j]) * w[j];
                    T arg = c;
#pragma unroll
                    for (int k = 0; k < D; ++k) arg = fma_t(Tk[k], P::off(off[k * n_pad + j]), arg);
                    acc = fma_t(P::ex2(arg), qq, acc);
                }
            }
        } else {
            for (int jb = 0; jb < TILE; jb += U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t j = j0 + jb + u;
                    T s = T(0);
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const T dd = t[k] - P::off(off[k * n_pad + j]);
                        s = fma_t(dd, dd, s);
                    }
                    acc = fma_t(P::ex2(-s), P::q(q[j]), acc);
                }
            }
        }
    }
    T *out = static_cast<T *>(a.out);
    if (a.splits == 1)
        out[i] = (i < a.n) ? acc + static_cast<T>(a.shift) * P::q(q[i]) : T(0);
    else
        out[static_cast<int64_t>(by) * n_pad + i] = acc;
}

// y_i = sum_s parts[s][i] + shift q_i for i < n, 0 on the padding.
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_kmvp_finish(int64_t n, int64_t n_pad, int splits, const void *parts_,
                                                       const void *q_, double shift, void *y_, const int *active) {
    if (active != nullptr && *active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    const T *parts = static_cast<const T *>(parts_);
    const typename P::Q *q = static_cast<const typename P::Q *>(q_);
    T *y = static_cast<T *>(y_);
    const int64_t i = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (i >= n_pad) return;
    if (i >= n) {
        y[i] = T(0);
        return;
    }
    T s = parts[i];
    for (int k = 1; k < splits; ++k) s += parts[static_cast<int64_t>(k) * n_pad + i];
    y[i] = s + static_cast<T>(shift) * P::q(q[i]);
}

KmvpPlan kmvp_plan(const Prepared &P, int prec) {
    (void)prec;
    KmvpPlan pl;
    const int rowblocks = P.ntiles;
    const int target_blocks = 4096;
    int splits = (target_blocks + rowblocks - 1) / rowblocks;
    int max_splits = P.ntiles / 2 > 1 ? P.ntiles / 2 : 1;
    if (splits > max_splits) splits = max_splits;
    if (splits < 1) splits = 1;
    pl.tiles_per_split = (P.ntiles + splits - 1) / splits;
    pl.splits = (P.ntiles + pl.tiles_per_split - 1) / pl.tiles_per_split;
    return pl;
}

size_t kmvp_parts_bytes(const Prepared &P, int prec) {
    const KmvpPlan pl = kmvp_plan(P, prec);
    const size_t el = prec == KRR_FP64 ? 8 : 4;
    return pl.splits > 1 ? static_cast<size_t>(pl.splits) * P.n_pad * el : 0;
}

template <int D, int PREC>
static hipError_t launch_kmvp(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_kmvp<D, PREC>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_kmvp_d(int dpad, const KArgs &a, hipStream_t s) {
    switch (dpad) {
        case 1: return launch_kmvp<1, PREC>(a, s);
        case 2: return launch_kmvp<2, PREC>(a, s);
        case 3: return launch_kmvp<3, PREC>(a, s);
        case 4: return launch_kmvp<4, PREC>(a, s);
        case 6: return launch_kmvp<6, PREC>(a, s);
        case 8: return launch_kmvp<8, PREC>(a, s);
        case 12: return launch_kmvp<12, PREC>(a, s);
        case 16: return launch_kmvp<16, PREC>(a, s);
        case 24: return launch_kmvp<24, PREC>(a, s);
        case 32: return launch_kmvp<32, PREC>(a, s);
        case 48: return launch_kmvp<48, PREC>(a, s);
        case 64: return launch_kmvp<64, PREC>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t kmvp_sorted(const Prepared &P, int prec, double shift, const void *q, void *y, void *parts,
                       const int *active, hipStream_t s) {
    const KmvpPlan pl = kmvp_plan(P, prec);
    KArgs a;
    a.n = P.n;
    a.n_pad = P.n_pad;
    a.ntiles = P.ntiles;
    a.nrowblocks = P.ntiles;
    a.splits = pl.splits;
    a.tps = pl.tiles_per_split;
    a.anchor = P.anchor;
    a.tile_r2 = P.tile_r2;
    a.tile_nj = P.tile_nj;
    a.q = q;
    a.shift = shift;
    a.active = active;
    a.out = pl.splits > 1 ? parts : y;
    hipError_t e;
    switch (prec) {
        case KRR_FP64:
            a.off = P.off64;
            a.w = P.w64;
            e = launch_kmvp_d<KRR_FP64>(P.dpad, a, s);
            break;
        case KRR_FP32:
            a.off = P.off32;
            a.w = P.w32;
            e = launch_kmvp_d<KRR_FP32>(P.dpad, a, s);
            break;
        case KRR_BF16:
            a.off = P.off16;
            a.w = P.w16;
            e = launch_kmvp_d<KRR_BF16>(P.dpad, a, s);
            break;
        default: return hipErrorInvalidValue;
    }
    KRR_HIP(e);
    if (pl.splits > 1) {
        const dim3 g((P.n_pad + BLOCK - 1) / BLOCK);
        switch (prec) {
            case KRR_FP64:
                hipLaunchKernelGGL(k_kmvp_finish<KRR_FP64>, g, dim3(BLOCK), 0, s, P.n, P.n_pad, pl.splits, parts, q,
                                   shift, y, active);
                break;
            case KRR_FP32:
                hipLaunchKernelGGL(k_kmvp_finish<KRR_FP32>, g, dim3(BLOCK), 0, s, P.n, P.n_pad, pl.splits, parts, q,
                                   shift, y, active);
                break;
            default:
                hipLaunchKernelGGL(k_kmvp_finish<KRR_BF16>, g, dim3(BLOCK), 0, s, P.n, P.n_pad, pl.splits, parts, q,
                                   shift, y, active);
                break;
        }
        KRR_HIP(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace krr
