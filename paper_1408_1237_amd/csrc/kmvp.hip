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
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "krr_internal.h"
#include "split16.h"

namespace krr {

// Block order: the hardware deals consecutive block ids round-robin to the 8
// XCDs, and the products keep that order (block id = row tile + row tiles x
// column split).  Their source data is a few MB (it sits in every XCD's L2
// either way) and they are bound by arithmetic, so the round-robin deal, which
// spreads dense and sparse row tiles over all XCDs, beats giving each XCD a
// contiguous range of row tiles: measured 4-5% faster on uniform points and
// 14-16% on clustered ones, whose row tiles carry very different work.

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Lane k's value of v (k a wave-uniform index), as a scalar.
__device__ __forceinline__ double lane_value(double v, int k) {
    const uint64_t bits = __builtin_bit_cast(uint64_t, v);
    const unsigned lo = __builtin_amdgcn_readlane(static_cast<unsigned>(bits), k);
    const unsigned hi = __builtin_amdgcn_readlane(static_cast<unsigned>(bits >> 32), k);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

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
    using Off = float;  // FP32 values, BF16-rounded on compact tiles (prep)
    using Q = uint16_t;
    static constexpr double wide = WIDE_R2_FP32;
    static __device__ __forceinline__ T off(Off v) { return v; }
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

// Rows are the target points (one lane each), columns the source points.  For
// the square product both are the same prepared set and the shift term is added.
struct KArgs {
    int64_t n_rows, n_pad_rows;  // targets
    int nrowblocks;
    const double *row_anchor;
    const void *row_off;
    int64_t n_pad;               // sources
    int ntiles, splits, tps;     // tps: tiles per block, a multiple of gtiles
    int gtiles, ngroups;         // column tiles per partial-sum group, groups
    const double *anchor;
    const double *tile_r2;
    const double *tile_nj;
    const float *tile_far;       // split-f16 kernel: per-tile far threshold on |t|^2
    const float *tile_far64;     // FP64 matrix-core kernel: the same for exponents <= -1100
    const void *slots;           // split-f16 kernel: source slot octets of the product's precision
    const void *off;
    const void *pm;  // point-major offsets (dpad > 16)
    const double *sq;  // |o_j|^2 of the FP64 offsets (Matern matrix-core form)
    const void *q;
    const void *qw;  // q_j * w_j in the arithmetic type (folded tiles)
    const void *w;   // w_j in the arithmetic type (symmetric product: the source terms)
    int zmem;        // symmetric product: 1 adds the source terms into the slots in memory even
                     // where the column group fits in LDS (the two paths are bitwise equal)
    void *out;
    double shift;    // square products only
    int square;
    const int *active;
    const double *row_r2;             // targets: squared radius of each row tile (far-tile skipping)
    unsigned long long *skip_count;   // when profiling: += row-tile rows x column tiles skipped as far
};

// A row tile (anchor aI, radius rI) and a column tile (anchor aJ) whose every
// pair is beyond the column tile's far threshold far_t2 on |t|^2 = |x_i - aJ|^2:
// |x_i - aJ| >= |aI - aJ| - rI for every target, so when (|aI - aJ| - rI)^2
// exceeds far_t2 (with a 1e-6 margin for the rounding of both sides) each
// target of the row tile would take the far clamp against the whole column
// tile, whose pairs then contribute exactly zero (exp2 underflows in the
// product's precision; also on wide tiles, whose direct exponents are then
// <= -200, or -1100 in FP64).  The products skip such tile pairs.
template <int D>
__device__ __forceinline__ bool tiles_far(const double (&aI)[D], double rI, const double *__restrict__ aJ,
                                          float far_t2) {
    double dd = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double v = aI[k] - aJ[k];
        dd = __builtin_fma(v, v, dd);
    }
    const double gap = sqrt(dd) - rI;
    return gap > 0.0 && gap * gap > 1.000001 * static_cast<double>(far_t2) + 1e-6;
}

template <int D, int PREC>
// The source arrays and the output are separate noalias kernel arguments: the
// group partial sums are stored inside the tile loop, and only non-aliasing
// arguments let the compiler keep the wave-uniform source reads on the scalar
// unit.
__global__ __launch_bounds__(BLOCK) void k_kmvp(KArgs a, const typename Prec<PREC>::Off *__restrict__ off,
                                                const typename Prec<PREC>::T *__restrict__ qw,
                                                const double *__restrict__ anchor,
                                                typename Prec<PREC>::T *__restrict__ out) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    using Q = typename P::Q;
    using Off = typename P::Off;
    constexpr int U = unroll_cols<D, PREC>();
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const int64_t n_pad = a.n_pad;

    const int lb = static_cast<int>(blockIdx.x);
    const int bx = lb % a.nrowblocks, by = lb / a.nrowblocks;
    const int64_t i = static_cast<int64_t>(bx) * BLOCK + threadIdx.x;
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);

    double aI[D];
    T oi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        aI[k] = a.row_anchor[static_cast<int64_t>(bx) * D + k];
        oi[k] = P::off(row_off[k * a.n_pad_rows + i]);
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
            // Source values of one chunk of U columns live in SGPRs; the next
            // chunk is requested before the current one is consumed.
            T co[D][U], cq[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cq[u] = qw[j0 + u];
#pragma unroll
                for (int k = 0; k < D; ++k) co[k][u] = P::off(off[k * n_pad + j0 + u]);
            }
            for (int jb = 0; jb < TILE; jb += U) {
                const int64_t jn = j0 + ((jb + U) & (TILE - 1));  // wraps on the last chunk (in bounds)
                T no[D][U], nq[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    nq[u] = qw[jn + u];
#pragma unroll
                    for (int k = 0; k < D; ++k) no[k][u] = P::off(off[k * n_pad + jn + u]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T arg = fma_t(Tk[0], co[0][u], c);
#pragma unroll
                    for (int k = 1; k < D; ++k) arg = fma_t(Tk[k], co[k][u], arg);
                    acc = fma_t(P::ex2(arg), cq[u], acc);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    cq[u] = nq[u];
#pragma unroll
                    for (int k = 0; k < D; ++k) co[k][u] = no[k][u];
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
        // close a partial-sum group (fixed tile ranges: the result does not
        // depend on how groups are dealt to blocks)
        if ((J + 1) % a.gtiles == 0 || J + 1 == J1) {
            if (a.ngroups == 1) {
                if (i < a.n_rows && a.square) acc += static_cast<T>(a.shift) * P::q(q[i]);
                out[i] = (i < a.n_rows) ? acc : T(0);
            } else {
                out[static_cast<int64_t>(J / a.gtiles) * a.n_pad_rows + i] = acc;
            }
            acc = T(0);
        }
    }
}

// ---------------------------------------------------------------- Matern kernel
//
// The Matern-3/2 product (eq. MaternKernel, section 6): with coordinates scaled
// by sqrt(3) / h the kernel of a pair is (1 + s) e^(-s), s = ||x~_i - x~_j||.
// One lane per target row; per pair d differences and FMAs for s^2, one square
// root, one exp2 (of -s log2 e) and two FMAs; sources at wave-uniform addresses
// (scalar loads), partial sums over fixed column-tile groups as in k_kmvp.
template <int D, int PREC>
__global__ __launch_bounds__(BLOCK) void k_kmvp_matern(KArgs a, const typename Prec<PREC>::Off *__restrict__ off,
                                                       const typename Prec<PREC>::Q *__restrict__ q,
                                                       const double *__restrict__ anchor,
                                                       typename Prec<PREC>::T *__restrict__ out) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    using Off = typename P::Off;
    constexpr int U = unroll_cols<D, PREC>();
    constexpr double LOG2E = 1.4426950408889634074;
    const int64_t n_pad = a.n_pad;
    const int lb = static_cast<int>(blockIdx.x);
    const int bx = lb % a.nrowblocks, by = lb / a.nrowblocks;
    const int64_t i = static_cast<int64_t>(bx) * BLOCK + threadIdx.x;
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    double aI[D];
    T oi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        aI[k] = a.row_anchor[static_cast<int64_t>(bx) * D + k];
        oi[k] = P::off(row_off[k * a.n_pad_rows + i]);
    }
    T acc = T(0);
    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    for (int J = J0; J < J1; ++J) {
        T t[D];
#pragma unroll
        for (int k = 0; k < D; ++k)
            t[k] = static_cast<T>((aI[k] - anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(oi[k]));
        const int64_t j0 = static_cast<int64_t>(J) * TILE;
        for (int jb = 0; jb < TILE; jb += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = j0 + jb + u;
                T r2 = T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const T dd = t[k] - P::off(off[k * n_pad + j]);
                    r2 = fma_t(dd, dd, r2);
                }
                const T sd = sqrt(r2);
                const T e = P::ex2(-sd * static_cast<T>(LOG2E));
                acc = fma_t(fma_t(sd, e, e), P::q(q[j]), acc);
            }
        }
        if ((J + 1) % a.gtiles == 0 || J + 1 == J1) {
            if (a.ngroups == 1) {
                if (i < a.n_rows && a.square) acc += static_cast<T>(a.shift) * P::q(q[i]);
                out[i] = (i < a.n_rows) ? acc : T(0);
            } else {
                out[static_cast<int64_t>(J / a.gtiles) * a.n_pad_rows + i] = acc;
            }
            acc = T(0);
        }
    }
}

// ---------------------------------------------------------------- VALU form, d = 24 .. 64
//
// The VALU products of k_kmvp (Gaussian) and k_kmvp_matern for the large
// compiled dimensions, with the same arithmetic in the same order per pair (the
// results are bitwise those of the small-d kernels' loops).  The small-d
// kernels keep the d coordinates of a group of columns in scalar registers,
// reached through d coordinate addresses, with the row anchors beside them; at
// d >= 24 that overflows the scalar register file.  Here the sources come from
// the point-major copy pm ([n_pad][D]): a group of UC columns is one contiguous
// run read by scalar loads at immediate offsets from a single base, two
// columns at a time; the anchor differences of a tile sit one coordinate per
// lane (read out with readlane) and the target offsets are re-read per tile
// through a pointer that advances one coordinate per load behind an empty
// statement (otherwise the compiler forms all d addresses up front in scalar
// registers).
template <int D, int PREC, bool MAT>
__global__ __launch_bounds__(BLOCK) void k_kmvp_hd(KArgs a, const typename Prec<PREC>::Off *__restrict__ pm,
                                                   const typename Prec<PREC>::T *__restrict__ qw,
                                                   const double *__restrict__ anchor,
                                                   typename Prec<PREC>::T *__restrict__ out) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    using Q = typename P::Q;
    using Off = typename P::Off;
    constexpr int UC = 16;  // columns per group
    // a group is read in chunks of KCH coordinates of a column pair (32 scalar
    // registers), software-pipelined one chunk ahead
    constexpr int KCH = (PREC == KRR_FP64 || D % 16 != 0) ? 8 : 16;
    constexpr int NKC = D / KCH;          // chunks per column pair
    constexpr int NCK = (UC / 2) * NKC;   // chunks per group
    // the FP64 Matern product (direct form only) measured faster with the
    // column pairs left to the compiler's scheduling
    constexpr bool PIPE = !(MAT && PREC == KRR_FP64);
    static_assert(D % KCH == 0, "whole chunks per column");
    auto load_chunk = [&](const typename Prec<PREC>::Off *b, int ck, typename Prec<PREC>::Off *dst) {
        const int u = 2 * (ck / NKC), k0 = (ck % NKC) * KCH;
#pragma unroll
        for (int e = 0; e < KCH; ++e) {
            dst[e] = b[u * D + k0 + e];
            dst[KCH + e] = b[(u + 1) * D + k0 + e];
        }
    };
    static_assert(D <= WAVE && TILE % UC == 0, "one anchor coordinate per lane; whole groups per tile");
    constexpr double LOG2E = 1.4426950408889634074;
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const int lb = static_cast<int>(blockIdx.x);
    const int bx = lb % a.nrowblocks, by = lb / a.nrowblocks;
    const int64_t i = static_cast<int64_t>(bx) * BLOCK + threadIdx.x;
    const int lane = threadIdx.x % WAVE;
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    const double aB = lane < D ? a.row_anchor[static_cast<int64_t>(bx) * D + lane] : 0.0;

    T acc = T(0);
    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    for (int J = J0; J < J1; ++J) {
        const double dA = lane < D ? aB - anchor[static_cast<int64_t>(J) * D + lane] : 0.0;
        // t_k = x_k - a_Jk of this lane's target, kept as 2 t_k
        T Tk[D];
        double tt = 0.0;
        {
            const Off *rp = row_off + i;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T tk = static_cast<T>(lane_value(dA, k) + static_cast<double>(P::off(*rp)));
                rp += a.n_pad_rows;
                asm volatile("" : "+v"(rp));
                Tk[k] = tk + tk;
                tt = __builtin_fma(static_cast<double>(tk), static_cast<double>(tk), tt);
            }
        }
        const int64_t j0 = static_cast<int64_t>(J) * TILE;
        const bool folded = !MAT && a.tile_r2[J] <= P::wide;
        const T init = folded ? static_cast<T>(-tt - a.tile_nj[J]) : T(0);
        for (int jb = 0; jb < TILE; jb += UC) {
            // per column: folded, the exponent c + sum_k 2 t_k o_k; direct, the
            // squared distance sum_k (t_k - o_k)^2
            const Off *cb = pm + (j0 + jb) * D;
            T arg[UC];
            if constexpr (PIPE) {
                T a0 = init, a1 = init, dep = init;
                Off cur[2 * KCH];
                load_chunk(cb, 0, cur);
#pragma unroll
                for (int ck = 0; ck < NCK; ++ck) {
                    const int u = 2 * (ck / NKC), k0 = (ck % NKC) * KCH;
                    Off nxt[2 * KCH];
                    if (ck + 1 < NCK) {
                        // the next chunk's loads wait for the previous chunk's
                        // arithmetic (through dep): two chunks in flight at most
                        // (a zero index that the compiler cannot see through: the
                        // address stays based on pm, whose reads may then use the
                        // scalar unit, and readfirstlane marks it uniform again)
                        int z = 0;
                        asm volatile("" : "+s"(z) : "v"(dep));
                        load_chunk(cb + __builtin_amdgcn_readfirstlane(z), ck + 1, nxt);
                    }
                    if (k0 == 0) a0 = a1 = init;
#pragma unroll
                    for (int e = 0; e < KCH; ++e) {
                        const T tk2 = Tk[k0 + e];
                        if (folded) {
                            a0 = fma_t(tk2, P::off(cur[e]), a0);
                            a1 = fma_t(tk2, P::off(cur[KCH + e]), a1);
                        } else {
                            const T tk = tk2 * T(0.5);
                            const T d0 = tk - P::off(cur[e]);
                            const T d1 = tk - P::off(cur[KCH + e]);
                            a0 = fma_t(d0, d0, a0);
                            a1 = fma_t(d1, d1, a1);
                        }
                    }
                    if (k0 + KCH == D) {
                        arg[u] = a0;
                        arg[u + 1] = a1;
                    }
                    dep = a0;
#pragma unroll
                    for (int e = 0; e < 2 * KCH; ++e) cur[e] = nxt[e];
                }
            } else {
#pragma unroll
                for (int u = 0; u < UC; u += 2) {
                    T a0 = init, a1 = init;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const T tk = Tk[k] * T(0.5);
                        const T d0 = tk - P::off(cb[u * D + k]);
                        const T d1 = tk - P::off(cb[(u + 1) * D + k]);
                        a0 = fma_t(d0, d0, a0);
                        a1 = fma_t(d1, d1, a1);
                    }
                    arg[u] = a0;
                    arg[u + 1] = a1;
                }
            }
            if (folded) {
#pragma unroll
                for (int u = 0; u < UC; ++u) acc = fma_t(P::ex2(arg[u]), qw[j0 + jb + u], acc);
            } else {
#pragma unroll
                for (int u = 0; u < UC; ++u) {
                    const int64_t j = j0 + jb + u;
                    if (MAT) {
                        const T sd = sqrt(arg[u]);
                        const T e = P::ex2(-sd * static_cast<T>(LOG2E));
                        acc = fma_t(fma_t(sd, e, e), P::q(q[j]), acc);
                    } else {
                        acc = fma_t(P::ex2(-arg[u]), P::q(q[j]), acc);
                    }
                }
            }
        }
        // close a partial-sum group
        if ((J + 1) % a.gtiles == 0 || J + 1 == J1) {
            if (a.ngroups == 1) {
                if (i < a.n_rows && a.square) acc += static_cast<T>(a.shift) * P::q(q[i]);
                out[i] = (i < a.n_rows) ? acc : T(0);
            } else {
                out[static_cast<int64_t>(J / a.gtiles) * a.n_pad_rows + i] = acc;
            }
            acc = T(0);
        }
    }
}

// ---------------------------------------------------------------- matrix-core exponent
//
// Products with the exponent on the matrix cores.  The folded exponent of a
// pair is an inner product of length d + 1,
//   arg_ij = [2 t_i, c_i] . [o_j, 1],   t_i = x_i - a_J, c_i = -||t_i||^2 - N_J,
// so one v_mfma_{f32,f64}_16x16x4 per 4 coordinates (DK = ceil((d+1)/4) of
// them) forms it for 16 x 16 pairs at once: A = the 16 sources x 4 coordinates
// (one value per lane: row l % 16, coordinate l / 16 of the chunk), B = the 4
// coordinates x 16 targets (lane l: target l % 16).  The accumulator gives lane
// l target l % 16 against four sources: rows 4 (l / 16) + v of the block in FP32,
// rows l / 16 + 4 v in FP64; for FP64 the A rows hold the sources in the order
// 0, 4, 8, 12, 1, 5, ... so that the four sources of lane l are 4 (l / 16) + v in
// both precisions (their q w values are then one contiguous 4-vector).  The VALU
// does exp2 and one fused multiply-add per pair, accumulating each target's sum in
// the four lanes that hold it (added by two cross-lane steps at the end).  A wave
// owns 4 groups of 16 targets (64 rows), a block one 256-row tile.  Wide tiles
// use the direct form on the VALU.
typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

template <int PREC>
struct MG;
template <>
struct MG<KRR_FP64> {
    using T = double;
    using V4 = doublex4_t;
    static constexpr bool permute_rows = true;
    static __device__ __forceinline__ V4 mfma(T a, T b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ T fma(T a, T b, T c) { return __builtin_fma(a, b, c); }
};
template <>
struct MG<KRR_FP32> {
    using T = float;
    using V4 = floatx4_t;
    static constexpr bool permute_rows = false;
    static __device__ __forceinline__ V4 mfma(T a, T b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ T fma(T a, T b, T c) { return __builtin_fmaf(a, b, c); }
};
template <>
struct MG<KRR_BF16> : MG<KRR_FP32> {};


// Groups of 16 targets per wave: 4 (a block covers one 256-row tile), or 2
// for FP64 at d = 16, where four groups' accumulators and operands do not fit
// two waves per SIMD (a block then covers half a tile; measured 10% faster
// there, 6% slower at d = 12).
template <int D, int PREC>
constexpr int mg_groups() {
    return (PREC == KRR_FP64 && D >= 16) ? 2 : 4;
}

template <int D, int PREC>
__global__ __launch_bounds__(BLOCK) void k_kmvp_mg(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using M = MG<PREC>;
    using T = typename M::T;
    using V4 = typename M::V4;
    using Off = typename P::Off;
    using Q = typename P::Q;
    constexpr int DK = (D + 4) / 4;  // chunks of 4 over the d + 1 coordinates
    constexpr int RG = mg_groups<D, PREC>();  // groups of 16 targets per wave
    constexpr int HB = 4 / RG;                // blocks per 256-row tile
    // LDS holds the d offset rows; coordinate d (the constant 1) and the zero
    // padding up to 4 DK are formed in registers (at d = 16 FP64 the four extra
    // rows would cost the second block per CU)
    constexpr int LDO = TILE + 16;  // padded LDS row: coordinate rows start 16 banks apart
    // The sources of the current column tile (offsets, and q w on folded tiles or
    // q on wide ones) are staged in LDS, double-buffered: the block loads tile
    // J + 1 from memory while it computes tile J.
    __shared__ T s_off[2][D][LDO];
    __shared__ __align__(16) T s_q[2][TILE];
    // FP64: the table of 2^(j/N) (exp2_tab): N = 4096 (32 KiB; a degree-2
    // polynomial, two FMAs fewer per pair than N = 256, relative error 2.5e-14,
    // far below the 1e-12 bar of the products) at d <= 3; N = 256 above (larger
    // tables measured no faster there, and at d = 4 the compiler then gave up a
    // wave per SIMD)
    constexpr bool TAB = PREC == KRR_FP64;
    constexpr int TN = D <= 3 ? 4096 : 256;
    __shared__ double s_exp2[TAB ? TN : 1];
    if constexpr (TAB) {
        for (int k = threadIdx.x; k < TN; k += BLOCK) s_exp2[k] = TN == 256 ? EXP2_TABLE256[k] : EXP2_TABLE4096[k];
    }
    const Off *__restrict__ off = static_cast<const Off *>(a.off);
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const T *__restrict__ qw = static_cast<const T *>(a.qw);
    const int64_t n_pad = a.n_pad;

    const int nrb = a.nrowblocks * HB;
    const int lb = static_cast<int>(blockIdx.x);
    const int bh = lb % nrb, by = lb / nrb;
    const int bx = bh / HB;  // row tile
    const int tid = threadIdx.x;
    const int lane = tid % WAVE;
    const int r16 = lane % 16, g = lane / 16;
    // source of A row r16 within a 16-column step
    const int asrc = M::permute_rows ? (r16 % 4) * 4 + r16 / 4 : r16;
    const int64_t row0 = static_cast<int64_t>(bx) * BLOCK + (bh % HB) * (BLOCK / HB) + (tid / WAVE) * (16 * RG);

    double aI[D];
#pragma unroll
    for (int k = 0; k < D; ++k) aI[k] = a.row_anchor[static_cast<int64_t>(bx) * D + k];
    // the lane's target offsets stay in registers when they fit in 64 VGPRs (32
    // with two groups), else they are re-read once per column tile
    constexpr bool KEEP = RG * D * sizeof(T) <= (RG == 2 ? 128 : 256);
    T oi[KEEP ? RG : 1][KEEP ? D : 1];
    if constexpr (KEEP) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
            for (int k = 0; k < D; ++k) oi[rg][k] = P::off(row_off[k * a.n_pad_rows + row0 + rg * 16 + r16]);
    }
    T acc[RG];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) acc[rg] = T(0);
    T *__restrict__ out = static_cast<T *>(a.out);

    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    // staging registers: this thread's source of the next tile
    T st_o[D], st_q;
    auto stage_load = [&](int J) {
        const int64_t j = static_cast<int64_t>(J) * TILE + tid;
#pragma unroll
        for (int k = 0; k < D; ++k) st_o[k] = P::off(off[k * n_pad + j]);
        st_q = a.tile_r2[J] > P::wide ? static_cast<T>(P::q(q[j])) : qw[j];
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < D; ++k) s_off[buf][k][tid] = st_o[k];
        s_q[buf][tid] = st_q;
    };
    // close partial-sum group grp (fixed tile ranges: the result does not
    // depend on how groups are dealt to blocks, nor on which tiles are skipped)
    auto close_group = [&](int grp) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            T sum = acc[rg];
            sum += __shfl_xor(sum, 16, WAVE);
            sum += __shfl_xor(sum, 32, WAVE);
            acc[rg] = T(0);
            const int64_t i = row0 + rg * 16 + r16;
            if (g == 0) {
                if (a.ngroups == 1) {
                    if (i < a.n_rows && a.square) sum += static_cast<T>(a.shift) * P::q(q[i]);
                    out[i] = (i < a.n_rows) ? sum : T(0);
                } else {
                    out[static_cast<int64_t>(grp) * a.n_pad_rows + i] = sum;
                }
            }
        }
    };
    // only the column tiles not far from this row tile (tiles_far; FP64: the
    // -1100 threshold) are staged and computed; groups without one get zero sums
    const double rI = a.row_r2 != nullptr ? sqrt(a.row_r2[bx]) : INFINITY;  // null: no skipping
    const float *__restrict__ far_t = TAB ? a.tile_far64 : a.tile_far;
    auto next_live = [&](int J) {
        while (J < J1 && tiles_far<D>(aI, rI, a.anchor + static_cast<int64_t>(J) * D, far_t[J])) ++J;
        return J;
    };
    const int gt = a.gtiles, g_last = (J1 - 1) / gt;
    int J = next_live(J0);
    int skipped = J - J0;
    for (int grp = J0 / gt; grp < (J < J1 ? J / gt : g_last + 1); ++grp) close_group(grp);
    if (J < J1) {
        stage_load(J);
        stage_store(0);
    }
    __syncthreads();
    int buf = 0;
    while (J < J1) {
        const int Jn = next_live(J + 1);
        skipped += Jn - J - 1;
        if (Jn < J1) stage_load(Jn);
        const double r2 = a.tile_r2[J];
        const double nj = a.tile_nj[J];
        // t = x - a_J of target group rg's lane (below d = 16 not kept over the
        // folded path: the wide path forms it again)
        auto target_t = [&](int rg, T (&t)[D]) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                T o;
                if constexpr (KEEP)
                    o = oi[rg][k];
                else
                    o = P::off(row_off[k * a.n_pad_rows + row0 + rg * 16 + r16]);
                t[k] = static_cast<T>((aI[k] - a.anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(o));
            }
        };
        // at d = 16 with four groups keeping t for the wide path (formed in the
        // same loop as |t|^2) measured faster than forming it again
        constexpr bool KEEP_T = D >= 16 && RG == 4;
        T t_keep[KEEP_T ? RG : 1][KEEP_T ? D : 1];
        T bval[RG][DK];
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            T t[D];
            double tt = 0.0;
            if constexpr (KEEP_T) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    T o;
                    if constexpr (KEEP)
                        o = oi[rg][k];
                    else
                        o = P::off(row_off[k * a.n_pad_rows + row0 + rg * 16 + r16]);
                    t_keep[rg][k] = static_cast<T>((aI[k] - a.anchor[static_cast<int64_t>(J) * D + k]) +
                                                   static_cast<double>(o));
                    const double tk = static_cast<double>(t_keep[rg][k]);
                    tt = __builtin_fma(tk, tk, tt);
                    t[k] = t_keep[rg][k];
                }
            } else {
                target_t(rg, t);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double tk = static_cast<double>(t[k]);
                    tt = __builtin_fma(tk, tk, tt);
                }
            }
            T c = static_cast<T>(-tt - nj);
            // FP64: the operand is scaled by N (exactly) for exp2_tab, and a
            // target whose every exponent against the tile is <= -1100 (exp2 is
            // 0 in FP64 either way) gets -2000 for the whole tile, which keeps
            // the scaled exponents in int range
            const T sc = TAB ? T(TN) : T(1);
            bool far = false;
            if constexpr (TAB) {
                far = tt > static_cast<double>(a.tile_far64[J]);
                c = far ? T(-2000.0 * TN) : c * sc;
            }
            // coordinate 4 kc + g of [2t, c, 0...] for this lane's chunk slots
#pragma unroll
            for (int kc = 0; kc < DK; ++kc) {
                const int dim = 4 * kc + g;
                T v = (dim == D) ? c : T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) v = (dim == k) ? (far ? T(0) : T(2) * sc * t[k]) : v;
                bval[rg][kc] = v;
            }
        }
        if (r2 <= P::wide) {
            // Software pipeline over the 16 column steps of the tile: the matrix
            // cores form the exponents of step cb + 16 (own accumulators) while
            // the VALU exponentiates and accumulates step cb.
            auto load_step = [&](int cb, T (&av)[DK], V4 &qv) {
#pragma unroll
                for (int kc = 0; kc < DK; ++kc) {
                    const int dim = 4 * kc + g;
                    if (4 * kc + 3 < D) {
                        av[kc] = s_off[buf][dim][cb + asrc];
                    } else {
                        // the last chunk: offsets below d, then the constant 1 and zeros
                        // (as o * [dim < d] + [dim == d])
                        const T o = s_off[buf][min(dim, D - 1)][cb + asrc];
                        av[kc] = M::fma(o, static_cast<T>(dim < D), static_cast<T>(dim == D));
                    }
                }
                qv = *reinterpret_cast<const V4 *>(&s_q[buf][cb + 4 * g]);
            };
            auto exponents = [&](const T (&av)[DK], V4 (&G)[RG]) {
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    G[rg] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
                    for (int kc = 0; kc < DK; ++kc) G[rg] = M::mfma(av[kc], bval[rg][kc], G[rg]);
                }
            };
            auto accumulate = [&](const V4 (&G)[RG], const V4 &qv) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg) {
                        if constexpr (TAB)
                            acc[rg] = M::fma(exp2_tab<TN>(G[rg][v], s_exp2), qv[v], acc[rg]);
                        else
                            acc[rg] = M::fma(P::ex2(G[rg][v]), qv[v], acc[rg]);
                    }
            };
            // 16 column steps, fully unrolled with two register sets so the
            // pipeline needs no copies
            T av[2][DK];
            V4 qv[2], G[2][RG];
            load_step(0, av[0], qv[0]);
            exponents(av[0], G[0]);
#pragma unroll
            for (int st = 1; st < TILE / 16; ++st) {
                load_step(st * 16, av[st & 1], qv[st & 1]);
                exponents(av[st & 1], G[st & 1]);
                accumulate(G[(st - 1) & 1], qv[(st - 1) & 1]);
            }
            accumulate(G[(TILE / 16 - 1) & 1], qv[(TILE / 16 - 1) & 1]);
        } else {
            T t[RG][D];
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                if constexpr (KEEP_T) {
#pragma unroll
                    for (int k = 0; k < D; ++k) t[rg][k] = t_keep[rg][k];
                } else {
                    target_t(rg, t[rg]);
                }
            }
            for (int cb = 0; cb < TILE; cb += 16) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int cj = cb + 4 * g + v;
                    T oc[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) oc[k] = s_off[buf][k][cj];
                    const T qj = s_q[buf][cj];
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg) {
                        T ss = T(0);
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const T dd = t[rg][k] - oc[k];
                            ss = M::fma(dd, dd, ss);
                        }
                        acc[rg] = M::fma(P::ex2(-ss), qj, acc[rg]);
                    }
                }
            }
        }
        const int gend = Jn < J1 ? Jn / gt : g_last + 1;
        for (int grp = J / gt; grp < gend; ++grp) close_group(grp);
        if (Jn < J1) stage_store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
        J = Jn;
    }
    if (a.skip_count != nullptr && tid == 0 && skipped > 0)
        atomicAdd(a.skip_count, static_cast<unsigned long long>(skipped) * (BLOCK / HB));
}

// ---------------------------------------------------------------- symmetric FP64 product
//
// K_hat is symmetric, so one exponential serves both of its terms: k_ij q_j in
// y_i and k_ij q_i in y_j.  The tiles are cut into groups of gs = a.gtiles
// consecutive tiles; block (R, C), R <= C, takes the tile pairs (I, J) with I
// in group R, J in group C and I < J, evaluating each pair once for both
// directions, plus on the diagonal (R == C) the tiles I == J one-sided.  The
// exponents are those of k_kmvp_mg with the operands exchanged: the targets
// form the A operand of v_mfma_f64_16x16x4f64 (rows in the order 0, 4, 8, 12,
// 1, 5, ...) and the sources the B operand, so lane l holds source l % 16 of
// the step against targets 4 (l / 16) + v of each target group.  The terms
// for the targets then accumulate per lane over the whole column loop (summed
// over the 16 source lanes once per row tile); those for the sources are
// summed per step over the lane's 16 targets, over the 4 lane rows by two
// cross-lane steps and over the 4 waves in LDS once per tile pair.  On folded
// tiles the exponent lacks the source factor w_j = 2^(N_J - |o_j|^2), which the
// source terms take once per tile pair (the target terms read q_j w_j).
//
// Partial sums: slot g of row i (a.out[g n_pad + i], a.ngroups slots) is
// written by exactly one block: for i in group X, block (X, g) when g > X (its
// target terms), block (g, X) when g < X (its source terms) and block (X, X)
// (both).  A block clears its source-side slots first; every later change of
// an entry comes from the thread that cleared it, so the sums are formed in a
// fixed order, independent of the launch.
// v + v of lane l ^ 32 (v_permlane32_swap on both halves of the double): the
// same sum, in the same order, in both lanes
__device__ __forceinline__ double join64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}
__device__ __forceinline__ double sum_halves32(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = static_cast<unsigned>(b), hi = static_cast<unsigned>(b >> 32);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return join64(l[0], h[0]) + join64(l[1], h[1]);
}
// v + v of lane l ^ 16 (v_permlane16_swap: rows of 16 lanes), likewise
__device__ __forceinline__ double sum_rows16(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = static_cast<unsigned>(b), hi = static_cast<unsigned>(b >> 32);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return join64(l[0], h[0]) + join64(l[1], h[1]);
}

// Largest group (tiles) of the symmetric product's launch (kmvp_sym_group_tiles
// stays below it up to 6.7e7 points).
constexpr int MS_MAX_GROUP_TILES = 512;

template <int D>
constexpr bool ms_supported() {
    return D <= 16;
}

// Tiles of a column group whose source terms k_kmvp_ms keeps in LDS: what fits
// beside its other LDS arrays within 76 KiB (two blocks per CU), at most 16.
template <int D, bool MAT>
constexpr int ms_zacc_tiles() {
    const int nbuf = D >= 16 ? 1 : 2, tn = (D <= 3 && !MAT) ? 4096 : 256;
    const int other = nbuf * D * (TILE + 16) * 8 + nbuf * TILE * 8 * (MAT ? 2 : 1) + tn * 8 +
                      (BLOCK / WAVE) * TILE * 8 + 512;
    const int t = (76 * 1024 - other) / (TILE * 8);
    return t > 16 ? 16 : (t < 1 ? 1 : t);
}

template <int D, bool MAT>
__global__ __launch_bounds__(BLOCK, 2) void k_kmvp_ms(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using M = MG<KRR_FP64>;
    using T = double;
    using V4 = doublex4_t;
    // chunks of 4 over the d + 1 coordinates [o, 1] (Matern: d + 2, [o, 1, |o'|^2])
    constexpr int DK = (D + (MAT ? 5 : 4)) / 4;
    constexpr double L2E = 1.4426950408889634074, LN2 = 0.69314718055994530942;
    // groups of 16 targets per wave: 4 (a block takes a row tile at once), or
    // 2 at d = 16, where four groups' operands and accumulators do not fit (a
    // block then takes a row tile in two units of 128 rows); there the source
    // tile is also staged in one buffer (two would leave one block per CU)
    constexpr int RG = D >= 16 ? 2 : 4;
    constexpr int UNITS = 4 / RG;
    constexpr int NBUF = D >= 16 ? 1 : 2;
    constexpr int NW = BLOCK / WAVE;
    constexpr int LDO = TILE + 16;
    // exp2_tab table (as k_kmvp_mg; Matern: the 256-entry one, which leaves room
    // for its staged source constants within two blocks per CU)
    constexpr int TN = (D <= 3 && !MAT) ? 4096 : 256;
    // target offsets kept in registers at small d, else re-read per tile pair
    constexpr bool KEEP = D <= 4;
    __shared__ T s_off[NBUF][D][LDO];
    __shared__ __align__(16) T s_q[NBUF][TILE];
    __shared__ double s_exp2[TN];
    // per wave: the source terms of the current tile pair (and, at the end of a
    // row tile, the block's target terms)
    __shared__ T s_z[NW * TILE];
    // the column tiles of group C not far from the current row tile
    __shared__ unsigned char s_live[MS_MAX_GROUP_TILES];
    // the source terms of group C, when it fits (entry [jl][j] owned by thread j)
    constexpr int ZMAX = ms_zacc_tiles<D, MAT>();
    __shared__ T s_zacc[ZMAX][TILE];
    // Matern: the sources' log2(e)^2 |o|^2 (the prepared FP64 squares)
    __shared__ T s_e[MAT ? NBUF : 1][MAT ? TILE : 1];
    for (int k = threadIdx.x; k < TN; k += BLOCK) s_exp2[k] = TN == 256 ? EXP2_TABLE256[k] : EXP2_TABLE4096[k];
    const T *__restrict__ off = static_cast<const T *>(a.off);
    const T *__restrict__ row_off = static_cast<const T *>(a.row_off);
    const T *__restrict__ q = static_cast<const T *>(a.q);
    const T *__restrict__ qw = static_cast<const T *>(a.qw);
    const T *__restrict__ wsrc = static_cast<const T *>(a.w);
    T *__restrict__ out = static_cast<T *>(a.out);
    const int64_t n_pad = a.n_pad;
    const int ng = a.ngroups, gs = a.gtiles;

    // block -> group pair (R, C): the ng (ng - 1) / 2 off-diagonal pairs first
    // (row-major over R < C; pair row R starts at R (2 ng - R - 1) / 2), then
    // the ng diagonal ones, which carry about half the work.  Consecutive
    // blocks go to different XCDs: where far tile pairs are skipped the work
    // sits near the diagonal, a few blocks of every row, and contiguous ranges
    // per XCD (rows of very different lengths) would load them unevenly.
    const int nb_off = ng * (ng - 1) / 2;
    const int b = blockIdx.x;
    int R, C;
    if (b < nb_off) {
        const double m = 2.0 * ng - 1.0;
        int r = static_cast<int>(0.5 * (m - sqrt(m * m - 8.0 * b)));
        r = r < 0 ? 0 : (r > ng - 2 ? ng - 2 : r);
        while (r > 0 && r * (2 * ng - r - 1) / 2 > b) --r;
        while ((r + 1) * (2 * ng - r - 2) / 2 <= b) ++r;
        R = r;
        C = r + 1 + (b - r * (2 * ng - r - 1) / 2);
    } else {
        R = C = b - nb_off;
    }
    const bool diag = R == C;
    const int tid = threadIdx.x;
    const int lane = tid % WAVE, wv = tid / WAVE;
    const int r16 = lane % 16, g = lane / 16;
    const int asrc = (r16 % 4) * 4 + r16 / 4;  // target of A row r16 within a group of 16
    const int I0 = R * gs, I1 = min(a.ntiles, I0 + gs);
    const int C0 = C * gs, C1 = min(a.ntiles, C0 + gs);
    T *__restrict__ zslot = out + static_cast<int64_t>(R) * n_pad;  // source terms of the tiles of group C
    T *__restrict__ yslot = out + static_cast<int64_t>(C) * n_pad;  // target terms of the tiles of group R
    // the source terms accumulate in LDS and are stored once (a group that
    // does not fit adds them into its cleared slots in memory instead)
    const bool zlds = a.zmem == 0 && C1 - C0 <= ZMAX;
    for (int J = C0; J < C1; ++J) {
        if (zlds)
            s_zacc[J - C0][tid] = T(0);
        else
            zslot[static_cast<int64_t>(J) * TILE + tid] = T(0);
    }

    T st_o[D], st_q, st_e = T(0);
    auto stage_load = [&](int J) {
        const int64_t j = static_cast<int64_t>(J) * TILE + tid;
#pragma unroll
        for (int k = 0; k < D; ++k) st_o[k] = off[k * n_pad + j];
        if constexpr (MAT) {
            st_q = q[j];  // no folded weights
            st_e = static_cast<T>(L2E * L2E) * a.sq[j];
        } else {
            st_q = a.tile_r2[J] > WIDE_R2_FP64 ? q[j] : qw[j];
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < D; ++k) s_off[buf][k][tid] = st_o[k];
        s_q[buf][tid] = st_q;
        if constexpr (MAT) s_e[buf][tid] = st_e;
    };
    // the source terms of one step (lane-local sum zl over the lane's targets):
    // summed over the 4 lane rows (the same sum, in the same order, in each;
    // all four lanes store it)
    auto emit_z = [&](T zl, int cb) {
        zl = sum_halves32(sum_rows16(zl));
        s_z[wv * TILE + cb + r16] = zl;
    };
    int skipped = 0;
    for (int I = I0; I < I1; ++I) {
        double aI[D];
#pragma unroll
        for (int k = 0; k < D; ++k) aI[k] = a.row_anchor[static_cast<int64_t>(I) * D + k];
        const double rI = a.row_r2 != nullptr ? sqrt(a.row_r2[I]) : INFINITY;  // null: no skipping
        // which column tiles are live: one thread per tile
        const int Js = diag ? I : C0;
        for (int jj = tid; jj < C1 - Js; jj += BLOCK) {
            const int Jt = Js + jj;
            s_live[jj] = tiles_far<D>(aI, rI, a.anchor + static_cast<int64_t>(Jt) * D, a.tile_far64[Jt]) ? 0 : 1;
        }
        __syncthreads();
        auto next_live = [&](int J) {
            while (J < C1 && s_live[J - Js] == 0) ++J;
            return J;
        };
        const int Jfirst = next_live(Js);
        skipped += Jfirst - Js;
        if (Jfirst >= C1) {
            // no live column tile: zero target terms (the source-side slots stay as they are)
            const int64_t i = static_cast<int64_t>(I) * TILE + tid;
            if (!diag) yslot[i] = T(0);
            __syncthreads();  // s_live is rewritten for the next row tile
            continue;
        }
        for (int unit = 0; unit < UNITS; ++unit) {
        const int64_t row0 = static_cast<int64_t>(I) * TILE + unit * (TILE / UNITS) + wv * (16 * RG);
        int J = Jfirst;
        T oi[KEEP ? RG : 1][KEEP ? D : 1];
        if constexpr (KEEP) {
#pragma unroll
            for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                for (int k = 0; k < D; ++k) oi[rg][k] = row_off[k * a.n_pad_rows + row0 + rg * 16 + asrc];
        }
        // q of the lane's output targets (unweighted; 0 on the padding)
        V4 qt[RG], acc[RG];
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = row0 + rg * 16 + 4 * g + v;
                qt[rg][v] = i < a.n_rows ? q[i] : T(0);
            }
            acc[rg] = V4{T(0), T(0), T(0), T(0)};
        }
        {
            stage_load(J);
            stage_store(0);
        }
        __syncthreads();
        int buf = 0;
        while (J < C1) {
            const int Jn = next_live(J + 1);
            if (unit == 0) skipped += Jn - J - 1;
            if (Jn < C1) stage_load(Jn);
            const double r2 = a.tile_r2[J];
            const double nj = a.tile_nj[J];
            const double *__restrict__ aJ = a.anchor + static_cast<int64_t>(J) * D;
            auto tile = [&](auto sym_c) {
                constexpr bool SYM = decltype(sym_c)::value;
                if (r2 <= WIDE_R2_FP64) {
                    // A operand: [2t, c, 0...] of target asrc(r16) of group rg, scaled by TN
                    T bval[RG][DK];
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg) {
                        T t[D];
                        double tt = 0.0;
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            T o;
                            if constexpr (KEEP)
                                o = oi[rg][k];
                            else
                                o = row_off[k * a.n_pad_rows + row0 + rg * 16 + asrc];
                            t[k] = (aI[k] - aJ[k]) + o;
                            tt = __builtin_fma(t[k], t[k], tt);
                        }
                        if constexpr (MAT) {
                            // [-2 log2(e)^2 t, log2(e)^2 |t|^2, 1]: the product forms
                            // (log2(e) s)^2 (as k_kmvp_mgw; far pairs reach the exponential's
                            // clamp)
#pragma unroll
                            for (int kc = 0; kc < DK; ++kc) {
                                const int dim = 4 * kc + g;
                                T v = (dim == D) ? static_cast<T>(L2E * L2E) * tt : (dim == D + 1 ? T(1) : T(0));
#pragma unroll
                                for (int k = 0; k < D; ++k) v = (dim == k) ? static_cast<T>(-2.0 * L2E * L2E) * t[k] : v;
                                bval[rg][kc] = v;
                            }
                        } else {
                            // a target whose every exponent against the tile is <= -1100
                            // gets -2000 for the whole tile (exp2 is 0 either way)
                            const bool far = tt > static_cast<double>(a.tile_far64[J]);
                            const T c = far ? T(-2000.0 * TN) : (-tt - nj) * T(TN);
#pragma unroll
                            for (int kc = 0; kc < DK; ++kc) {
                                const int dim = 4 * kc + g;
                                T v = (dim == D) ? c : T(0);
#pragma unroll
                                for (int k = 0; k < D; ++k) v = (dim == k) ? (far ? T(0) : T(2 * TN) * t[k]) : v;
                                bval[rg][kc] = v;
                            }
                        }
                    }
                    auto load_step = [&](int cb, T (&av)[DK], T &qs) {
#pragma unroll
                        for (int kc = 0; kc < DK; ++kc) {
                            const int dim = 4 * kc + g;
                            if (4 * kc + 3 < D) {
                                av[kc] = s_off[buf][dim][cb + r16];
                            } else {
                                const T o = s_off[buf][min(dim, D - 1)][cb + r16];
                                av[kc] = M::fma(o, static_cast<T>(dim < D), static_cast<T>(dim == D));
                                if constexpr (MAT) av[kc] = M::fma(s_e[buf][cb + r16], static_cast<T>(dim == D + 1), av[kc]);
                            }
                        }
                        qs = s_q[buf][cb + r16];
                    };
                    auto exponents = [&](const T (&av)[DK], V4 (&G)[RG]) {
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg) {
                            G[rg] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
                            for (int kc = 0; kc < DK; ++kc) G[rg] = M::mfma(bval[rg][kc], av[kc], G[rg]);
                        }
                    };
                    auto accumulate = [&](const V4 (&G)[RG], T qs, int cb) {
                        T zl[RG];  // independent chains, one per target group
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg) zl[rg] = T(0);
#pragma unroll
                        for (int v = 0; v < 4; ++v)
#pragma unroll
                            for (int rg = 0; rg < RG; ++rg) {
                                // the pair's kernel value: 2^G (folded Gaussian, G scaled by
                                // TN), or the Matern 2^-u (1 + u ln2), u = sqrt(G)
                                T e;
                                if constexpr (MAT) {
                                    const T u = __builtin_sqrt(__builtin_fabs(G[rg][v]));
                                    e = exp2_tab<TN>(__builtin_fmax(-u * TN, -2000.0 * TN), s_exp2) *
                                        M::fma(u, static_cast<T>(LN2), T(1));
                                } else {
                                    e = exp2_tab<TN>(G[rg][v], s_exp2);
                                }
                                acc[rg][v] = M::fma(e, qs, acc[rg][v]);
                                if constexpr (SYM) zl[rg] = M::fma(e, qt[rg][v], zl[rg]);
                            }
                        if constexpr (SYM) {
                            T zs = zl[0];
#pragma unroll
                            for (int rg = 1; rg < RG; ++rg) zs += zl[rg];
                            emit_z(zs, cb);
                        }
                    };
                    // software pipeline over the 16 column steps (as k_kmvp_mg)
                    T av[2][DK], qs[2];
                    V4 G[2][RG];
                    load_step(0, av[0], qs[0]);
                    exponents(av[0], G[0]);
#pragma unroll
                    for (int st = 1; st < TILE / 16; ++st) {
                        load_step(st * 16, av[st & 1], qs[st & 1]);
                        exponents(av[st & 1], G[st & 1]);
                        accumulate(G[(st - 1) & 1], qs[(st - 1) & 1], (st - 1) * 16);
                    }
                    accumulate(G[(TILE / 16 - 1) & 1], qs[(TILE / 16 - 1) & 1], TILE - 16);
                } else {
                    // wide tile: the direct form, in chunks of 4 column steps, one
                    // output target at a time (few registers: wide tiles are rare)
#pragma unroll 1
                    for (int ch = 0; ch < TILE / 64; ++ch) {
                        T zs[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll 1
                        for (int rv = 0; rv < 4 * RG; ++rv) {
                            // at d = 16: keeps the staged offsets from being read once for
                            // all targets (registers the rest of the kernel needs; below,
                            // measured no better)
                            if constexpr (D >= 16) __asm__ __volatile__("" ::: "memory");
                            const int rg = rv / 4, v = rv % 4;
                            const int64_t i = row0 + rg * 16 + 4 * g + v;
                            T t[D];
#pragma unroll
                            for (int k = 0; k < D; ++k) t[k] = (aI[k] - aJ[k]) + row_off[k * a.n_pad_rows + i];
                            const T qi = i < a.n_rows ? q[i] : T(0);
                            T sacc = T(0);
#pragma unroll
                            for (int s4 = 0; s4 < 4; ++s4) {
                                const int cj = (4 * ch + s4) * 16 + r16;
                                T ss = T(0);
#pragma unroll
                                for (int k = 0; k < D; ++k) {
                                    const T dd = t[k] - s_off[buf][k][cj];
                                    ss = M::fma(dd, dd, ss);
                                }
                                T e;
                                if constexpr (MAT) {
                                    const T sd = __builtin_sqrt(ss);
                                    const T e0 = exp2_tab<TN>(__builtin_fmax(-L2E * sd * TN, -2000.0 * TN), s_exp2);
                                    e = M::fma(sd, e0, e0);
                                } else {
                                    e = exp2_tab<TN>(__builtin_fmax(-ss * TN, -2000.0 * TN), s_exp2);
                                }
                                sacc = M::fma(e, s_q[buf][cj], sacc);
                                if constexpr (SYM) zs[s4] = M::fma(e, qi, zs[s4]);
                            }
                            // into acc[rg][v] (rg, v vary at run time here)
#pragma unroll
                            for (int ra = 0; ra < RG; ++ra)
#pragma unroll
                                for (int va = 0; va < 4; ++va) acc[ra][va] += (ra == rg && va == v) ? sacc : T(0);
                        }
                        if constexpr (SYM) {
#pragma unroll
                            for (int s4 = 0; s4 < 4; ++s4) emit_z(zs[s4], (4 * ch + s4) * 16);
                        }
                    }
                }
            };
            const bool sym = J != I;
            // the slot entry this thread adds the tile pair's source terms to (its
            // own earlier store; read before the compute to hide the latency)
            const int64_t jz = static_cast<int64_t>(J) * TILE + tid;
            const T zold = (sym && !zlds) ? zslot[jz] : T(0);
            const T wj = (sym && r2 <= WIDE_R2_FP64 && !MAT) ? wsrc[jz] : T(1);  // Matern: no folding
            if (sym)
                tile(std::true_type{});
            else
                tile(std::false_type{});
            if constexpr (NBUF == 2) {
                if (Jn < C1) stage_store(buf ^ 1);
                __syncthreads();
            } else {
                __syncthreads();  // every wave is done with the staged tile
                if (Jn < C1) stage_store(0);
                if (!sym) __syncthreads();
            }
            if (sym) {
                // the tile pair's source terms: summed over the waves, times w_j on a folded tile
                const T z = (s_z[tid] + s_z[TILE + tid]) + (s_z[2 * TILE + tid] + s_z[3 * TILE + tid]);
                if (zlds)
                    s_zacc[J - C0][tid] += z * wj;
                else
                    zslot[jz] = zold + z * wj;
                __syncthreads();  // s_z is rewritten by the next tile pair (one buffer: the staging is visible)
            }
            if constexpr (NBUF == 2) buf ^= 1;
            J = Jn;
        }
        // the row tile's target terms: summed over the 16 source lanes; lane
        // column 0 holds targets rg 16 + 4 g + v of the wave
#pragma unroll
        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T x = acc[rg][v];
                x += __shfl_xor(x, 1, WAVE);
                x += __shfl_xor(x, 2, WAVE);
                x += __shfl_xor(x, 4, WAVE);
                x += __shfl_xor(x, 8, WAVE);
                acc[rg][v] = x;
            }
        if (r16 == 0) {
#pragma unroll
            for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                for (int v = 0; v < 4; ++v) s_z[wv * (16 * RG) + rg * 16 + 4 * g + v] = acc[rg][v];
        }
        __syncthreads();
        if (tid < TILE / UNITS) {
            const int il = unit * (TILE / UNITS) + tid;
            const int64_t i = static_cast<int64_t>(I) * TILE + il;
            if (!diag)
                yslot[i] = s_z[tid];
            else if (zlds)
                yslot[i] = s_z[tid] + s_zacc[I - C0][il];  // the source terms of tile I are complete
            else
                yslot[i] += s_z[tid];
        }
        __syncthreads();
        }  // unit
    }
    if (zlds && !diag) {
        for (int J = C0; J < C1; ++J) zslot[static_cast<int64_t>(J) * TILE + tid] = s_zacc[J - C0][tid];
    }
    // both directions of every skipped tile pair (rows x column tiles)
    if (a.skip_count != nullptr && tid == 0 && skipped > 0)
        atomicAdd(a.skip_count, static_cast<unsigned long long>(skipped) * 2 * TILE);
}

// ---------------------------------------------------------------- split-f16 matrix-core exponent
//
// FP32 and BF16 products with the folded exponent formed by the f16 matrix
// cores.  Every FP32 operand v is split as v = hi + lo, hi = f16(v),
// lo = f16(v - hi): |v - hi - lo| <= 2^-22 |v| (f16 subnormals are kept), four
// times the rounding of the FP32 operand itself.  The exponent of the form
// above becomes an inner product over 3d + 2 slots,
//   arg_ij = sum_k ( o_hi 2t_hi + o_hi 2t_lo + o_lo 2t_hi )_jk,ik + c_hi + c_lo,
// dropping only the lo * lo terms (at most 2^-22 of each product); the products
// are exact and accumulate in FP32 as in the FP32 matrix-core form.  One
// v_mfma_f32_32x32x16_f16 covers 32 sources x 32 targets x 16 slots.  Its lane
// layout: A (sources x slots) lane l holds source l % 32 and slots
// 8 (l / 32) .. + 7; B (slots x targets) lane l holds target l % 32 and the same
// slots; accumulator element v of lane l is source 8 (v / 4) + 4 (l / 32) + v % 4
// against target l % 32.  A wave owns 2 groups of 32 targets (64 rows).
//
// A target whose every pair with the tile has arg <= -200 (so that exp2 is 0 in
// FP32 either way) gets the exponent -2000 for the whole tile; the others have
// |c| < 640 and |2t| < 50 on tiles with R^2 <= 64, inside the f16 range.  Wide
// tiles (R^2 > 64, offsets possibly beyond the f16 range) are staged as plain
// FP32 offsets in the same LDS words and take the direct form.
//
// MAT: the Matern-3/2 product.  With t' = log2(e) t and o' = log2(e) o the
// same operation forms G = |t'|^2 + |o'|^2 - 2 t'.o' = (log2(e) s)^2 (the
// source constant |o'|^2 is prepared with the slots); per pair the VALU takes
// u = sqrt(|G|), e = exp2(-u) and accumulates e (q + u ln2 q) = (1 + s) e^-s q
// (ln2 q staged beside q).  A target at scaled distance >= 111 from every source
// of a tile (exp2 is 0 in FP32) gets G = 60000 for the tile; the others have
// |t'|^2 < 30000 and |2t'| < 350, inside the f16 range.
typedef float floatx16_t __attribute__((ext_vector_type(16)));

// Lane l of a wave holds values of target (l / 32, l % 32); v_permlane32_swap
// exchanges the upper half of its first operand with the lower half of its
// second.  Given a lane's lo and hi values, g0 receives lo of target (0, l % 32)
// in lanes 0-31 and hi of it in lanes 32-63, g1 the same for target (1, l % 32):
// the B operands of both target groups from one operand build per lane.
__device__ __forceinline__ void swap_halves(half8_t lo, half8_t hi, half8_t &g0, half8_t &g1) {
    const uintx4_t L = __builtin_bit_cast(uintx4_t, lo), H = __builtin_bit_cast(uintx4_t, hi);
    uintx4_t A, B;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const unsigned le = L[e], he = H[e];
        const auto r = __builtin_amdgcn_permlane32_swap(le, he, false, false);
        A[e] = r[0];
        B[e] = r[1];
    }
    g0 = __builtin_bit_cast(half8_t, A);
    g1 = __builtin_bit_cast(half8_t, B);
}
// The same for one value per lane: g0 = v of target (0, l % 32), g1 = v of (1, l % 32).
__device__ __forceinline__ void swap_halves(float v, float &g0, float &g1) {
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    g0 = __builtin_bit_cast(float, static_cast<unsigned>(r[0]));
    g1 = __builtin_bit_cast(float, static_cast<unsigned>(r[1]));
}

template <int D, int PREC, bool MAT>
__global__ __launch_bounds__(BLOCK) void k_kmvp_mh(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using Off = typename P::Off;
    using Q = typename P::Q;
    constexpr int KC = split_chunks(D);  // 16-slot chunks (3D + 4 slots: Gaussian and Matern forms)
    static_assert(KC >= 1 && 16 * KC >= 3 * D + 4, "slot chunks cover the split inner product");
    constexpr int RG = 2;               // groups of 32 targets per wave
    static_assert(P::wide <= 64.0, "the f16 range bound assumes R^2 <= 64 on folded tiles");
    // sources of the current column tile, double-buffered: their slot vectors
    // ([buffer][chunk * 2 + half][source], 8 slots each) and q w (or q on wide
    // tiles; Matern: q, and ln2 q in s_q2)
    __shared__ __align__(16) half8_t s_a[2][2 * KC][TILE];
    __shared__ __align__(16) float s_q[2][TILE];
    __shared__ __align__(16) float s_q2[MAT ? 2 : 1][MAT ? TILE : 4];
    const Off *__restrict__ off = static_cast<const Off *>(a.off);
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const float *__restrict__ qw = static_cast<const float *>(a.qw);
    const int64_t n_pad = a.n_pad;

    const int lb = static_cast<int>(blockIdx.x);
    const int bx = lb % a.nrowblocks, by = lb / a.nrowblocks;
    const int tid = threadIdx.x;
    const int lane = tid % WAVE;
    const int r32 = lane % 32, h = lane / 32;
    const int64_t row0 = static_cast<int64_t>(bx) * BLOCK + (tid / WAVE) * 64;

    double aI[D];
#pragma unroll
    for (int k = 0; k < D; ++k) aI[k] = a.row_anchor[static_cast<int64_t>(bx) * D + k];
    // lane l forms the target operand of row row0 + l (group l / 32, target
    // l % 32) and trades half of it with lane l ^ 32 (see swap_halves)
    float oi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) oi[k] = P::off(row_off[k * a.n_pad_rows + row0 + lane]);
    float acc[RG];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) acc[rg] = 0.f;
    float *__restrict__ out = static_cast<float *>(a.out);

    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    // staging registers: this thread's source of the next tile, its slot octets
    // (prepared with the points) or, on wide tiles, its plain FP32 offsets
    // (coordinate k in word k % 4 of octet k / 4)
    const half8_t *__restrict__ slots = static_cast<const half8_t *>(a.slots);
    half8_t st_a[2 * KC];
    float st_q;
    auto stage_load = [&](int J) {
        const int64_t j = static_cast<int64_t>(J) * TILE + tid;
        if (a.tile_r2[J] > P::wide) {
#pragma unroll
            for (int c = 0; c < 2 * KC; ++c) {
                uintx4_t u;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float o = (4 * c + e < D) ? P::off(off[(4 * c + e) * n_pad + j]) : 0.f;
                    u[e] = __builtin_bit_cast(unsigned, o);
                }
                st_a[c] = __builtin_bit_cast(half8_t, u);
            }
            st_q = P::q(q[j]);
        } else {
#pragma unroll
            for (int c = 0; c < 2 * KC; ++c) st_a[c] = slots[c * n_pad + j];
            st_q = MAT ? P::q(q[j]) : qw[j];
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < 2 * KC; ++c) s_a[buf][c][tid] = st_a[c];
        s_q[buf][tid] = st_q;
        if constexpr (MAT) s_q2[buf][tid] = LN2_F * st_q;
    };
    // close partial-sum group grp (fixed tile ranges: the result does not
    // depend on how groups are dealt to blocks, nor on which tiles are skipped)
    auto close_group = [&](int grp) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            float sum = acc[rg];
            sum += __shfl_xor(sum, 32, WAVE);
            acc[rg] = 0.f;
            const int64_t i = row0 + rg * 32 + r32;
            if (h == 0) {
                if (a.ngroups == 1) {
                    if (i < a.n_rows && a.square) sum += static_cast<float>(a.shift) * P::q(q[i]);
                    out[i] = (i < a.n_rows) ? sum : 0.f;
                } else {
                    out[static_cast<int64_t>(grp) * a.n_pad_rows + i] = sum;
                }
            }
        }
    };
    // only the column tiles not far from this row tile (tiles_far) are staged
    // and computed; groups without one get zero sums
    const double rI = a.row_r2 != nullptr ? sqrt(a.row_r2[bx]) : INFINITY;  // null: no skipping
    auto next_live = [&](int J) {
        while (J < J1 && tiles_far<D>(aI, rI, a.anchor + static_cast<int64_t>(J) * D, a.tile_far[J])) ++J;
        return J;
    };
    const int gt = a.gtiles, g_last = (J1 - 1) / gt;
    int J = next_live(J0);
    int skipped = J - J0;
    for (int grp = J0 / gt; grp < (J < J1 ? J / gt : g_last + 1); ++grp) close_group(grp);
    if (J < J1) {
        stage_load(J);
        stage_store(0);
    }
    __syncthreads();
    int buf = 0;
    while (J < J1) {
        const int Jn = next_live(J + 1);
        skipped += Jn - J - 1;
        if (Jn < J1) stage_load(Jn);
        const double r2 = a.tile_r2[J];
        const float njf = static_cast<float>(a.tile_nj[J]);  // a small integer
        const float far_t2 = a.tile_far[J];
        // t = x - a_J of this lane's target
        float t[D];
        double tt = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double td = (aI[k] - a.anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(oi[k]);
            t[k] = static_cast<float>(td);
            tt = __builtin_fma(td, td, tt);
        }
        half8_t bval[RG][KC];
        if (r2 <= P::wide) {
            const bool far = static_cast<float>(tt) > far_t2;
            const _Float16 z16 = static_cast<_Float16>(0.f), one16 = static_cast<_Float16>(1.f);
            HiLo v[D], c, c2;
            if constexpr (MAT) {
                // -2 t', |t'|^2 (t' = log2(e) t) and the source constant's (1, 1)
#pragma unroll
                for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : -2.f * LOG2E_F * t[k]);
                c = far ? HiLo{static_cast<_Float16>(60000.f), z16}
                        : split_f16(LOG2E_F * LOG2E_F * static_cast<float>(tt));
                c2 = HiLo{one16, one16};
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : 2.f * t[k]);
                // c = -|t|^2 - N_J formed in FP32 (two roundings, 2^-23 relative)
                c = far ? HiLo{static_cast<_Float16>(-2000.f), z16} : split_f16(-static_cast<float>(tt) - njf);
                c2 = HiLo{z16, z16};
            }
            // this lane holds both octets of chunk kc for its own target; the B
            // operand wants octet h of targets (group 0, l % 32) and (group 1, l % 32)
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
                swap_halves(slot_octet<D, false>(2 * kc, v, c, c2), slot_octet<D, false>(2 * kc + 1, v, c, c2),
                            bval[0][kc], bval[1][kc]);
        }
        if (r2 <= P::wide) {
            // Software pipeline over the 8 column steps of 32 sources: the matrix
            // cores form step st (own accumulators) while the VALU exponentiates
            // and accumulates step st - 1; the source slots are read one step ahead.
            auto load_a = [&](int cb, half8_t (&av)[KC]) {
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) av[kc] = s_a[buf][2 * kc + h][cb + r32];
            };
            auto load_q = [&](int cb, floatx4_t (&qv)[4], floatx4_t (&qv2)[MAT ? 4 : 1]) {
#pragma unroll
                for (int m = 0; m < 4; ++m) qv[m] = *reinterpret_cast<const floatx4_t *>(&s_q[buf][cb + 8 * m + 4 * h]);
                if constexpr (MAT) {
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        qv2[m] = *reinterpret_cast<const floatx4_t *>(&s_q2[buf][cb + 8 * m + 4 * h]);
                }
            };
            auto exponents = [&](const half8_t (&av)[KC], floatx16_t (&G)[RG]) {
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) G[rg][v] = 0.f;
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc)
                        G[rg] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av[kc], bval[rg][kc], G[rg], 0, 0, 0);
                }
            };
            auto accumulate = [&](const floatx16_t (&G)[RG], const floatx4_t (&qv)[4],
                                  const floatx4_t (&qv2)[MAT ? 4 : 1]) {
                if constexpr (MAT || D < 16) {
#pragma unroll
                    for (int v = 0; v < 16; ++v)
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg) {
                            if constexpr (MAT) {
                                const float u = __builtin_amdgcn_sqrtf(__builtin_fabsf(G[rg][v]));
                                const float w = __builtin_fmaf(u, qv2[v / 4][v % 4], qv[v / 4][v % 4]);
                                acc[rg] = __builtin_fmaf(__builtin_amdgcn_exp2f(-u), w, acc[rg]);
                            } else {
                                acc[rg] = __builtin_fmaf(__builtin_amdgcn_exp2f(G[rg][v]), qv[v / 4][v % 4], acc[rg]);
                            }
                        }
                } else {
                    // D = 16: all exponentials of the step first, then the FMAs
                    // in the same order.  Written next to its FMA, each
                    // exponential was scheduled (at this kernel's register use)
                    // right before the FMA that reads it, with a wait state
                    // between them: 3 % of the kernel
                    floatx16_t E[RG];
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                        for (int v = 0; v < 16; ++v) E[rg][v] = __builtin_amdgcn_exp2f(G[rg][v]);
#pragma unroll
                    for (int v = 0; v < 16; ++v)
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg) acc[rg] = __builtin_fmaf(E[rg][v], qv[v / 4][v % 4], acc[rg]);
                }
            };
            half8_t av[2][KC];
            floatx4_t qv[4], qv2[MAT ? 4 : 1];
            floatx16_t G[2][RG];
            load_a(0, av[0]);
            exponents(av[0], G[0]);
            load_a(32, av[1]);
#pragma unroll
            for (int st = 1; st < TILE / 32; ++st) {
                exponents(av[st & 1], G[st & 1]);
                if (st + 1 < TILE / 32) load_a((st + 1) * 32, av[(st + 1) & 1]);
                load_q((st - 1) * 32, qv, qv2);
                accumulate(G[(st - 1) & 1], qv, qv2);
            }
            load_q((TILE / 32 - 1) * 32, qv, qv2);
            accumulate(G[(TILE / 32 - 1) & 1], qv, qv2);
        } else {
            // wide tile: the direct form sum_k (t_k - o_k)^2 on the VALU, the two
            // halves of the wave taking alternate sources (FP32 offsets staged)
            float tg[RG][D];  // t of targets (group 0, l % 32) and (group 1, l % 32)
#pragma unroll
            for (int k = 0; k < D; ++k) swap_halves(t[k], tg[0][k], tg[1][k]);
            for (int cs = 0; cs < TILE; cs += 2) {
                const int cj = cs + h;
                float oc[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    // the word goes through a scalar: a bit cast whose operand is a
                    // vector element reads the vector's first element in this compiler
                    const unsigned w = __builtin_bit_cast(uintx4_t, s_a[buf][k / 4][cj])[k % 4];
                    oc[k] = __builtin_bit_cast(float, w);
                }
                const float qj = s_q[buf][cj];
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    float ss = 0.f;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const float dd = tg[rg][k] - oc[k];
                        ss = __builtin_fmaf(dd, dd, ss);
                    }
                    if constexpr (MAT) {
                        const float sd = __builtin_sqrtf(ss);
                        const float e = __builtin_amdgcn_exp2f(-LOG2E_F * sd);
                        acc[rg] = __builtin_fmaf(__builtin_fmaf(sd, e, e), qj, acc[rg]);
                    } else {
                        acc[rg] = __builtin_fmaf(__builtin_amdgcn_exp2f(-ss), qj, acc[rg]);
                    }
                }
            }
        }
        const int gend = Jn < J1 ? Jn / gt : g_last + 1;
        for (int grp = J / gt; grp < gend; ++grp) close_group(grp);
        if (Jn < J1) stage_store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
        J = Jn;
    }
    if (a.skip_count != nullptr && tid == 0 && skipped > 0)
        atomicAdd(a.skip_count, static_cast<unsigned long long>(skipped) * BLOCK);
}

// v of the lane that DPP control C selects within its row of 16 (every row and
// bank written; each control used here has a source lane for every lane)
template <int C>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), C, 0xF, 0xF, true));
}

// ---------------------------------------------------------------- symmetric split-f16 product
//
// The FP32 / BF16 Gaussian product of k_kmvp_mh with one exponential per
// unordered pair, as k_kmvp_ms for FP64 (group pairs, tile pairs, partial-sum
// slots and their owners are the same).  The targets form the A operand of
// v_mfma_f32_32x32x16_f16 and the sources the B operand, so lane l holds source
// l % 32 of the step against targets 8 (v / 4) + 4 (l / 32) + v % 4 (v < 16)
// of the wave's 32 targets: the target terms accumulate per lane over the
// column loop (summed over the 32 source lanes once per row unit), the source
// terms are summed per step over the lane's 16 targets, over the two halves of
// the wave (v_permlane32_swap) and over the waves in LDS once per tile pair.
// A wave owns one group of 32 targets (two would keep twice the accumulators
// and target weights live and cost a wave per SIMD), so a block takes a row
// tile in two units of 128 rows, each against the same column tiles.  At
// d = 16 the source tiles are staged in one buffer (after a barrier that ends
// every wave's reads), which keeps two blocks per CU.
template <int D, int PREC, bool MAT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(D <= 4 ? 3 : 2))) void k_kmvp_mhs(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using Off = typename P::Off;
    using Q = typename P::Q;
    constexpr int KC = split_chunks(D);
    constexpr int NW = BLOCK / WAVE;
    constexpr int UNIT = NW * 32;  // rows per row unit
    static_assert(P::wide <= 64.0, "the f16 range bound assumes R^2 <= 64 on folded tiles");
    // one staging buffer at d = 16 (two would leave one block per CU)
    constexpr int NBUF = D >= 16 ? 1 : 2;
    __shared__ __align__(16) half8_t s_a[NBUF][2 * KC][TILE];
    __shared__ __align__(16) float s_q[NBUF][TILE];
    __shared__ float s_z[NW * TILE];
    __shared__ unsigned char s_live[MS_MAX_GROUP_TILES];
    // the source terms of group C, when it fits (entry [jl][j] owned by thread j;
    // 16 tiles keep the block within a third of the LDS)
    constexpr int ZMAX = 16;
    __shared__ float s_zacc[ZMAX][TILE];
    const Off *__restrict__ off = static_cast<const Off *>(a.off);
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const float *__restrict__ qw = static_cast<const float *>(a.qw);
    const float *__restrict__ wsrc = static_cast<const float *>(a.w);
    float *__restrict__ out = static_cast<float *>(a.out);
    const int64_t n_pad = a.n_pad;
    const int ng = a.ngroups, gs = a.gtiles;

    // block -> group pair (R, C), as k_kmvp_ms
    const int nb_off = ng * (ng - 1) / 2;
    const int b = blockIdx.x;
    int R, C;
    if (b < nb_off) {
        const double m = 2.0 * ng - 1.0;
        int r = static_cast<int>(0.5 * (m - sqrt(m * m - 8.0 * b)));
        r = r < 0 ? 0 : (r > ng - 2 ? ng - 2 : r);
        while (r > 0 && r * (2 * ng - r - 1) / 2 > b) --r;
        while ((r + 1) * (2 * ng - r - 2) / 2 <= b) ++r;
        R = r;
        C = r + 1 + (b - r * (2 * ng - r - 1) / 2);
    } else {
        R = C = b - nb_off;
    }
    const bool diag = R == C;
    const int tid = threadIdx.x;
    const int lane = tid % WAVE, wv = tid / WAVE;
    const int r32 = lane % 32, h = lane / 32;
    const int I0 = R * gs, I1 = min(a.ntiles, I0 + gs);
    const int C0 = C * gs, C1 = min(a.ntiles, C0 + gs);
    float *__restrict__ zslot = out + static_cast<int64_t>(R) * n_pad;
    float *__restrict__ yslot = out + static_cast<int64_t>(C) * n_pad;
    const bool zlds = a.zmem == 0 && C1 - C0 <= ZMAX;
    for (int J = C0; J < C1; ++J) {
        if (zlds)
            s_zacc[J - C0][tid] = 0.f;
        else
            zslot[static_cast<int64_t>(J) * TILE + tid] = 0.f;
    }

    // staging of a column tile's sources, as k_kmvp_mh
    const half8_t *__restrict__ slots = static_cast<const half8_t *>(a.slots);
    half8_t st_a[2 * KC];
    float st_q;
    auto stage_load = [&](int J) {
        const int64_t j = static_cast<int64_t>(J) * TILE + tid;
        if (a.tile_r2[J] > P::wide) {
#pragma unroll
            for (int c = 0; c < 2 * KC; ++c) {
                uintx4_t u;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float o = (4 * c + e < D) ? P::off(off[(4 * c + e) * n_pad + j]) : 0.f;
                    u[e] = __builtin_bit_cast(unsigned, o);
                }
                st_a[c] = __builtin_bit_cast(half8_t, u);
            }
            st_q = P::q(q[j]);
        } else {
#pragma unroll
            for (int c = 0; c < 2 * KC; ++c) st_a[c] = slots[c * n_pad + j];
            st_q = MAT ? P::q(q[j]) : qw[j];
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < 2 * KC; ++c) s_a[buf][c][tid] = st_a[c];
        s_q[buf][tid] = st_q;
    };
    // the source terms of one step: the lane-local sum over its targets, summed
    // over the two halves of the wave (the same sum in both) and stored
    auto emit_z = [&](float zl, int cb) {
        float z0, z1;
        swap_halves(zl, z0, z1);
        s_z[wv * TILE + cb + r32] = z0 + z1;
    };
    int skipped = 0;
    for (int I = I0; I < I1; ++I) {
        double aI[D];
#pragma unroll
        for (int k = 0; k < D; ++k) aI[k] = a.row_anchor[static_cast<int64_t>(I) * D + k];
        const double rI = a.row_r2 != nullptr ? sqrt(a.row_r2[I]) : INFINITY;  // null: no skipping
        const int Js = diag ? I : C0;
        for (int jj = tid; jj < C1 - Js; jj += BLOCK) {
            const int Jt = Js + jj;
            s_live[jj] = tiles_far<D>(aI, rI, a.anchor + static_cast<int64_t>(Jt) * D, a.tile_far[Jt]) ? 0 : 1;
        }
        __syncthreads();
        auto next_live = [&](int J) {
            while (J < C1 && s_live[J - Js] == 0) ++J;
            return J;
        };
        const int Jfirst = next_live(Js);
        skipped += Jfirst - Js;
        if (Jfirst >= C1) {
            const int64_t i = static_cast<int64_t>(I) * TILE + tid;
            if (!diag) yslot[i] = 0.f;
            __syncthreads();  // s_live is rewritten for the next row tile
            continue;
        }
        for (int half = 0; half < TILE / UNIT; ++half) {
            const int64_t row0 = static_cast<int64_t>(I) * TILE + half * UNIT + wv * 32;
            // the lane's A-operand target row0 + r32 (octet h of its slots)
            float oi[D];
#pragma unroll
            for (int k = 0; k < D; ++k) oi[k] = P::off(row_off[k * a.n_pad_rows + row0 + r32]);
            // the lane's output targets 8 (v / 4) + 4 h + v % 4: their q (0 on the
            // padding).  The product is square, so q is the sorted vector of n_pad
            // entries (as k_prescale reads it): the loads need no guard (a guard
            // made a branch per load), a select zeroes the padding
            float qt[16], acc[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t i = row0 + 8 * (v / 4) + 4 * h + v % 4;
                const float qi = P::q(q[i]);
                qt[v] = i < a.n_rows ? qi : 0.f;
                acc[v] = 0.f;
            }
            int J = Jfirst;
            stage_load(J);
            stage_store(0);
            __syncthreads();
            int buf = 0;
            while (J < C1) {
                const int Jn = next_live(J + 1);
                if (half == 0) skipped += Jn - J - 1;
                if (Jn < C1) stage_load(Jn);
                const double r2 = a.tile_r2[J];
                const float njf = static_cast<float>(a.tile_nj[J]);  // a small integer
                const float far_t2 = a.tile_far[J];
                const double *__restrict__ aJ = a.anchor + static_cast<int64_t>(J) * D;
                const bool sym = J != I;
                const int64_t jz = static_cast<int64_t>(J) * TILE + tid;
                const float zold = (sym && !zlds) ? zslot[jz] : 0.f;
                const float wj = (sym && r2 <= P::wide && !MAT) ? wsrc[jz] : 1.f;  // Matern: no folding
                auto tile = [&](auto sym_c) {
                    constexpr bool SYM = decltype(sym_c)::value;
                    if (r2 <= P::wide) {
                        // the target operand, as k_kmvp_mh's B operand
                        float t[D];
                        double tt = 0.0;
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const double td = (aI[k] - aJ[k]) + static_cast<double>(oi[k]);
                            t[k] = static_cast<float>(td);
                            tt = __builtin_fma(td, td, tt);
                        }
                        const bool far = static_cast<float>(tt) > far_t2;
                        const _Float16 z16 = static_cast<_Float16>(0.f), one16 = static_cast<_Float16>(1.f);
                        HiLo v[D], c, c2;
                        if constexpr (MAT) {
                            // -2 t', |t'|^2 and (1, 1) for the source constant, as k_kmvp_mh
#pragma unroll
                            for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : -2.f * LOG2E_F * t[k]);
                            c = far ? HiLo{static_cast<_Float16>(60000.f), z16}
                                    : split_f16(LOG2E_F * LOG2E_F * static_cast<float>(tt));
                            c2 = HiLo{one16, one16};
                        } else {
#pragma unroll
                            for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : 2.f * t[k]);
                            c = far ? HiLo{static_cast<_Float16>(-2000.f), z16}
                                    : split_f16(-static_cast<float>(tt) - njf);
                            c2 = HiLo{z16, z16};
                        }
                        half8_t tval[KC];
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc) {
                            const half8_t o0 = slot_octet<D, false>(2 * kc, v, c, c2);
                            const half8_t o1 = slot_octet<D, false>(2 * kc + 1, v, c, c2);
                            tval[kc] = h ? o1 : o0;
                        }
                        auto load_a = [&](int cb, half8_t (&av)[KC]) {
#pragma unroll
                            for (int kc = 0; kc < KC; ++kc) av[kc] = s_a[buf][2 * kc + h][cb + r32];
                        };
                        auto exponents = [&](const half8_t (&av)[KC], floatx16_t &G) {
#pragma unroll
                            for (int v2 = 0; v2 < 16; ++v2) G[v2] = 0.f;
#pragma unroll
                            for (int kc = 0; kc < KC; ++kc)
                                G = __builtin_amdgcn_mfma_f32_32x32x16_f16(tval[kc], av[kc], G, 0, 0, 0);
                        };
                        // the steps' source terms, stored to LDS after the last step (a
                        // store per step would hold up the next step's operand reads)
                        float zst[TILE / 32];
                        auto accumulate = [&](const floatx16_t &G, float qs, int st) {
                            float zl[4] = {0.f, 0.f, 0.f, 0.f};  // independent chains
#pragma unroll
                            for (int v2 = 0; v2 < 16; ++v2) {
                                // the pair's kernel value: 2^G (folded Gaussian), or the
                                // Matern (1 + s) e^-s = 2^-u (1 + u ln2), u = sqrt(G)
                                float e;
                                if constexpr (MAT) {
                                    const float u = __builtin_amdgcn_sqrtf(__builtin_fabsf(G[v2]));
                                    e = __builtin_amdgcn_exp2f(-u) * __builtin_fmaf(u, LN2_F, 1.f);
                                } else {
                                    e = __builtin_amdgcn_exp2f(G[v2]);
                                }
                                acc[v2] = __builtin_fmaf(e, qs, acc[v2]);
                                if constexpr (SYM) zl[v2 % 4] = __builtin_fmaf(e, qt[v2], zl[v2 % 4]);
                            }
                            if constexpr (SYM) {
                                float z0, z1;
                                swap_halves((zl[0] + zl[1]) + (zl[2] + zl[3]), z0, z1);
                                zst[st] = z0 + z1;
                            }
                        };
                        // software pipeline over the 8 column steps of 32 sources (as k_kmvp_mh)
                        half8_t av[2][KC];
                        floatx16_t G[2];
                        load_a(0, av[0]);
                        exponents(av[0], G[0]);
                        load_a(32, av[1]);
#pragma unroll
                        for (int st = 1; st < TILE / 32; ++st) {
                            exponents(av[st & 1], G[st & 1]);
                            if (st + 1 < TILE / 32) load_a((st + 1) * 32, av[(st + 1) & 1]);
                            accumulate(G[(st - 1) & 1], s_q[buf][(st - 1) * 32 + r32], st - 1);
                        }
                        accumulate(G[(TILE / 32 - 1) & 1], s_q[buf][TILE - 32 + r32], TILE / 32 - 1);
                        if constexpr (SYM) {
#pragma unroll
                            for (int st = 0; st < TILE / 32; ++st) s_z[wv * TILE + st * 32 + r32] = zst[st];
                        }
                    } else {
                        // wide tile: the direct form on the staged FP32 offsets, one
                        // output target at a time (few registers: wide tiles are rare)
                        float zs[TILE / 32];
#pragma unroll
                        for (int st = 0; st < TILE / 32; ++st) zs[st] = 0.f;
#pragma unroll 1
                        for (int v2 = 0; v2 < 16; ++v2) {
                            // keeps the staged offsets from being read once for all
                            // targets (registers the rest of the kernel needs)
                            __asm__ __volatile__("" ::: "memory");
                            const int64_t i = row0 + 8 * (v2 / 4) + 4 * h + v2 % 4;
                            float tg[D];
#pragma unroll
                            for (int k = 0; k < D; ++k)
                                tg[k] = static_cast<float>((aI[k] - aJ[k]) +
                                                           static_cast<double>(P::off(row_off[k * a.n_pad_rows + i])));
                            const float qi = i < a.n_rows ? P::q(q[i]) : 0.f;
                            float sacc = 0.f;
#pragma unroll
                            for (int st = 0; st < TILE / 32; ++st) {
                                const int cj = st * 32 + r32;
                                float ss = 0.f;
#pragma unroll
                                for (int k = 0; k < D; ++k) {
                                    // the word goes through a scalar (see k_kmvp_mh)
                                    const unsigned w = __builtin_bit_cast(uintx4_t, s_a[buf][k / 4][cj])[k % 4];
                                    const float dd = tg[k] - __builtin_bit_cast(float, w);
                                    ss = __builtin_fmaf(dd, dd, ss);
                                }
                                float e;
                                if constexpr (MAT) {
                                    const float sd = __builtin_sqrtf(ss);
                                    const float e0 = __builtin_amdgcn_exp2f(-LOG2E_F * sd);
                                    e = __builtin_fmaf(sd, e0, e0);
                                } else {
                                    e = __builtin_amdgcn_exp2f(-ss);
                                }
                                sacc = __builtin_fmaf(e, s_q[buf][cj], sacc);
                                if constexpr (SYM) zs[st] = __builtin_fmaf(e, qi, zs[st]);
                            }
                            // into acc[v2] (v2 varies at run time here)
#pragma unroll
                            for (int va = 0; va < 16; ++va) acc[va] += (va == v2) ? sacc : 0.f;
                        }
                        if constexpr (SYM) {
#pragma unroll
                            for (int st = 0; st < TILE / 32; ++st) emit_z(zs[st], st * 32);
                        }
                    }
                };
                if (sym)
                    tile(std::true_type{});
                else
                    tile(std::false_type{});
                if constexpr (NBUF == 2) {
                    if (Jn < C1) stage_store(buf ^ 1);
                    __syncthreads();
                } else {
                    __syncthreads();  // every wave is done with the one staging buffer
                    if (Jn < C1) stage_store(0);
                }
                if (sym) {
                    const float z = (s_z[tid] + s_z[TILE + tid]) + (s_z[2 * TILE + tid] + s_z[3 * TILE + tid]);
                    if (zlds)
                        s_zacc[J - C0][tid] = __builtin_fmaf(z, wj, s_zacc[J - C0][tid]);
                    else
                        zslot[jz] = __builtin_fmaf(z, wj, zold);
                }
                if (sym || NBUF == 1) __syncthreads();  // s_z rewritten next; the staging visible
                if constexpr (NBUF == 2) buf ^= 1;
                J = Jn;
            }
            // the unit's target terms, summed over the 32 source lanes of each
            // half: v_permlane16_swap pairs value v of the even row of 16 lanes
            // with value v + 8 of the odd row, so that after one add row parity
            // b holds value v + 8 b summed over both rows; four DPP adds then
            // sum each row (48 VALU operations against 80 lane permutes and 80
            // adds of a shuffle per value and stage)
            float red[8];
#pragma unroll
            for (int v2 = 0; v2 < 8; ++v2) {
                const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, acc[v2]),
                                                                __builtin_bit_cast(unsigned, acc[v2 + 8]), false, false);
                float x = __builtin_bit_cast(float, static_cast<unsigned>(r[0])) +
                          __builtin_bit_cast(float, static_cast<unsigned>(r[1]));
                x += dpp_f32<0x128>(x);  // row_ror:8, lane ^ 8
                x += dpp_f32<0x124>(x);  // row_ror:4: with the above, the lanes of one residue mod 4
                x += dpp_f32<0x4E>(x);   // quad_perm [2, 3, 0, 1]
                x += dpp_f32<0xB1>(x);   // quad_perm [1, 0, 3, 2]
                red[v2] = x;
            }
            if ((lane & 15) == 0) {
                const int b4 = (lane >> 4) & 1;
#pragma unroll
                for (int v2 = 0; v2 < 8; ++v2) {
                    const int v = v2 + 8 * b4;
                    s_z[wv * 32 + 8 * (v / 4) + 4 * h + v % 4] = red[v2];
                }
            }
            __syncthreads();
            if (tid < UNIT) {
                const int il = half * UNIT + tid;
                const int64_t i = static_cast<int64_t>(I) * TILE + il;
                if (!diag)
                    yslot[i] = s_z[tid];
                else if (zlds)
                    yslot[i] = s_z[tid] + s_zacc[I - C0][il];  // the source terms of tile I are complete
                else
                    yslot[i] += s_z[tid];
            }
            __syncthreads();
        }
    }
    if (zlds && !diag) {
        for (int J = C0; J < C1; ++J) zslot[static_cast<int64_t>(J) * TILE + tid] = s_zacc[J - C0][tid];
    }
    if (a.skip_count != nullptr && tid == 0 && skipped > 0)
        atomicAdd(a.skip_count, static_cast<unsigned long long>(skipped) * 2 * TILE);
}

// qw_j = q_j * w_j (the per-source factor of the folded form), once per product.
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_prescale(int64_t n_pad, const void *q_, const void *w_, void *qw_,
                                                    const int *active) {
    if (active != nullptr && *active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    const typename P::Q *q = static_cast<const typename P::Q *>(q_);
    const T *w = static_cast<const T *>(w_);
    T *qw = static_cast<T *>(qw_);
    const int64_t i = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (i < n_pad) qw[i] = P::q(q[i]) * w[i];
}

// y_i = sum_s parts[s][i] (+ shift q_i when square) for i < n, 0 on the padding.
// A block takes FINISH_ROWS<PREC> consecutive rows, 16 bytes of each slot per
// lane; wave w adds the slots w, w + 4, w + 8, ... in increasing order and the
// four wave sums are added in wave order, so the order is the same on every
// launch.  (One row per thread walking all slots left too few waves in flight
// to cover the latency of its dependent loads.)
template <int PREC>
constexpr int finish_rows() { return WAVE * static_cast<int>(16 / sizeof(typename Prec<PREC>::T)); }
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_kmvp_finish(int64_t n, int64_t n_pad, int ngroups, const void *parts_,
                                                       const void *q_, double shift, int square, void *y_,
                                                       const int *active) {
    if (active != nullptr && *active == 0) return;
    using P = Prec<PREC>;
    using T = typename P::T;
    constexpr int V = 16 / sizeof(T);
    constexpr int NW = BLOCK / WAVE;
    typedef T VT __attribute__((ext_vector_type(V)));
    __shared__ VT s_part[NW - 1][WAVE];
    const T *parts = static_cast<const T *>(parts_);
    const typename P::Q *q = static_cast<const typename P::Q *>(q_);
    T *y = static_cast<T *>(y_);
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int64_t i0 = blockIdx.x * static_cast<int64_t>(finish_rows<PREC>()) + lane * V;
    VT acc = {};
    if (i0 < n_pad) {  // n_pad is a multiple of V: the whole vector is inside
        const VT *p = reinterpret_cast<const VT *>(parts + i0);
        const int64_t stride = n_pad / V;
#pragma unroll 8
        for (int k = wv; k < ngroups; k += NW) acc += p[static_cast<int64_t>(k) * stride];
    }
    if (wv > 0) s_part[wv - 1][lane] = acc;
    __syncthreads();
    if (wv == 0 && i0 < n_pad) {
#pragma unroll
        for (int w = 0; w < NW - 1; ++w) acc += s_part[w][lane];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t i = i0 + v;
            y[i] = i >= n ? T(0) : square ? acc[v] + static_cast<T>(shift) * P::q(q[i]) : acc[v];
        }
    }
}

// ---------------------------------------------------------------- split-f16, d = 24 .. 48
//
// The split-f16 Gaussian product (FP32 / BF16) for the compiled dimensions 24,
// 32 and 48: the slots, operations and clamps of k_kmvp_mh, with 3D + 4 slots in
// KC = ceil((3D + 4) / 16) chunks.  Its operands do not fit the d <= 16 layout,
// so the sources of a column tile are staged in LDS 64 at a time (double
// buffered; a thread carries at most ceil(KC / 2) octets), the target operand
// is rebuilt once per column tile from the anchors and target offsets read
// from memory, and within a 64-source stage the matrix cores form the second
// 32-source step while the VALU exponentiates the first.  Wide tiles take the
// direct form on staged FP32 offsets, one target group at a time.
template <int D, int PREC, bool MAT>
__global__ __launch_bounds__(BLOCK) void k_kmvp_mhw(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using Off = typename P::Off;
    using Q = typename P::Q;
    constexpr int KC = split_chunks(D);
    constexpr int NOCT = 2 * KC;
    constexpr int RG = 2;                                  // groups of 32 targets per wave
    constexpr int CH = 64;                                 // sources per LDS stage
    constexpr int NCH = TILE / CH;                         // stages per column tile
    constexpr int NA = (NOCT * CH + BLOCK - 1) / BLOCK;    // octets staged per thread
    static_assert(KC >= 1 && 16 * KC >= 3 * D + 4 && TILE % CH == 0 && CH % 32 == 0, "stage layout");
    static_assert(P::wide <= 64.0, "the f16 range bound assumes R^2 <= 64 on folded tiles");
    __shared__ __align__(16) half8_t s_a[2][NOCT][CH];
    __shared__ __align__(16) float s_q[2][CH];
    __shared__ __align__(16) float s_q2[MAT ? 2 : 1][MAT ? CH : 4];
    const Off *__restrict__ off = static_cast<const Off *>(a.off);
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const float *__restrict__ qw = static_cast<const float *>(a.qw);
    const half8_t *__restrict__ slots = static_cast<const half8_t *>(a.slots);
    const int64_t n_pad = a.n_pad;

    const int lb = static_cast<int>(blockIdx.x);
    const int bx = lb % a.nrowblocks, by = lb / a.nrowblocks;
    const int tid = threadIdx.x;
    const int lane = tid % WAVE;
    const int r32 = lane % 32, h = lane / 32;
    const int64_t row0 = static_cast<int64_t>(bx) * BLOCK + (tid / WAVE) * 64;
    float acc[RG];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) acc[rg] = 0.f;
    float *__restrict__ out = static_cast<float *>(a.out);
    const half8_t zero8 = __builtin_bit_cast(half8_t, uintx4_t{0u, 0u, 0u, 0u});

    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    const int C0 = J0 * NCH, C1 = J1 * NCH;
    // staging: entry e = c * CH + col is octet c of source col of the stage; on
    // wide tiles octet c holds the FP32 offsets 4c .. 4c + 3
    half8_t st_a[NA];
    float st_q = 0.f;
    auto stage_load = [&](int ci) {
        const int J = ci / NCH;
        const int64_t j0 = static_cast<int64_t>(J) * TILE + (ci % NCH) * CH;
        const bool wide = a.tile_r2[J] > P::wide;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = u * BLOCK + tid;
            const int c = e / CH, col = e % CH;
            if (e >= NOCT * CH) {
                st_a[u] = zero8;
            } else if (wide) {
                uintx4_t v;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float o = (4 * c + i < D) ? P::off(off[(4 * c + i) * n_pad + j0 + col]) : 0.f;
                    v[i] = __builtin_bit_cast(unsigned, o);
                }
                st_a[u] = __builtin_bit_cast(half8_t, v);
            } else {
                st_a[u] = slots[c * n_pad + j0 + col];
            }
        }
        if (tid < CH) st_q = (wide || MAT) ? P::q(q[j0 + tid]) : qw[j0 + tid];
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = u * BLOCK + tid;
            if (e < NOCT * CH) s_a[buf][e / CH][e % CH] = st_a[u];
        }
        if (tid < CH) {
            s_q[buf][tid] = st_q;
            if constexpr (MAT) s_q2[buf][tid] = LN2_F * st_q;
        }
    };
    // the anchor difference a_B - a_J of the row block and tile J, coordinate
    // k in lane k (uniform values kept in vector registers: as scalars they
    // would not fit)
    auto anchor_diff = [&](int J) -> double {
        return lane < D ? a.row_anchor[static_cast<int64_t>(bx) * D + lane] - a.anchor[static_cast<int64_t>(J) * D + lane] : 0.0;
    };
    // the target's t = x - a_J for coordinates k = 0 .. D - 1 in turn: rp points
    // at coordinate k of the target's offsets and advances one coordinate per
    // call.  The empty statement keeps the pointer an opaque vector value, so
    // that the D coordinate addresses are not all formed up front in scalar
    // registers (which would not fit).
    auto target_t = [&](double dA, const Off *&rp, int k) -> double {
        const double td = lane_value(dA, k) + static_cast<double>(P::off(*rp));
        rp += a.n_pad_rows;
        asm volatile("" : "+v"(rp));
        return td;
    };

    if (C0 < C1) {
        stage_load(C0);
        stage_store(0);
    }
    __syncthreads();
    half8_t bval[RG][KC];
    for (int ci = C0; ci < C1; ++ci) {
        const int buf = (ci - C0) & 1;
        if (ci + 1 < C1) stage_load(ci + 1);
        const int J = ci / NCH;
        const bool wide = a.tile_r2[J] > P::wide;
        if (!wide && ci % NCH == 0) {
            // the target operand of tile J: 2t and c = -|t|^2 - N_J split as in k_kmvp_mh
            const float njf = static_cast<float>(a.tile_nj[J]);
            const float far_t2 = a.tile_far[J];
            // (lane l builds the operand of row row0 + l and trades half of it
            // with lane l ^ 32, as in k_kmvp_mh)
            const double dA = anchor_diff(J);
            float t[D];
            double tt = 0.0;
            const Off *rp = row_off + (row0 + lane);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double td = target_t(dA, rp, k);
                t[k] = static_cast<float>(td);
                tt = __builtin_fma(td, td, tt);
            }
            const bool far = static_cast<float>(tt) > far_t2;
            const _Float16 z16 = static_cast<_Float16>(0.f), one16 = static_cast<_Float16>(1.f);
            HiLo v[D], c, c2;
            if constexpr (MAT) {
                // -2 t', |t'|^2 (t' = log2(e) t) and the source constant's (1, 1)
#pragma unroll
                for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : -2.f * LOG2E_F * t[k]);
                c = far ? HiLo{static_cast<_Float16>(60000.f), z16}
                        : split_f16(LOG2E_F * LOG2E_F * static_cast<float>(tt));
                c2 = HiLo{one16, one16};
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : 2.f * t[k]);
                c = far ? HiLo{static_cast<_Float16>(-2000.f), z16} : split_f16(-static_cast<float>(tt) - njf);
                c2 = HiLo{z16, z16};
            }
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
                swap_halves(slot_octet<D, false>(2 * kc, v, c, c2), slot_octet<D, false>(2 * kc + 1, v, c, c2),
                            bval[0][kc], bval[1][kc]);
        }
        if (!wide) {
            // two 32-source steps, each one exponent block per target group on
            // the matrix cores followed by exp2 and the accumulation
#pragma unroll
            for (int st = 0; st < CH / 32; ++st) {
                floatx16_t G[RG];
                {
                    half8_t av[KC];
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) av[kc] = s_a[buf][2 * kc + h][st * 32 + r32];
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
                        for (int v = 0; v < 16; ++v) G[rg][v] = 0.f;
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc)
                            G[rg] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av[kc], bval[rg][kc], G[rg], 0, 0, 0);
                    }
                }
                floatx4_t qv[4], qv2[MAT ? 4 : 1];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    qv[m] = *reinterpret_cast<const floatx4_t *>(&s_q[buf][st * 32 + 8 * m + 4 * h]);
                    if constexpr (MAT) qv2[m] = *reinterpret_cast<const floatx4_t *>(&s_q2[buf][st * 32 + 8 * m + 4 * h]);
                }
                if constexpr (MAT) {
#pragma unroll
                    for (int v = 0; v < 16; ++v)
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg) {
                            // G = (log2(e) s)^2: (1 + s) e^(-s) q = 2^(-u) (q + u ln2 q), u = sqrt(G)
                            const float u = __builtin_amdgcn_sqrtf(__builtin_fabsf(G[rg][v]));
                            const float w = __builtin_fmaf(u, qv2[v / 4][v % 4], qv[v / 4][v % 4]);
                            acc[rg] = __builtin_fmaf(__builtin_amdgcn_exp2f(-u), w, acc[rg]);
                        }
                } else {
                    // exponentials first, then the FMAs in the same order (as
                    // k_kmvp_mh at D = 16: no wait state between each pair)
                    floatx16_t E[RG];
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                        for (int v = 0; v < 16; ++v) E[rg][v] = __builtin_amdgcn_exp2f(G[rg][v]);
#pragma unroll
                    for (int v = 0; v < 16; ++v)
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg) acc[rg] = __builtin_fmaf(E[rg][v], qv[v / 4][v % 4], acc[rg]);
                }
            }
        } else {
            // wide tile: the direct form on the staged FP32 offsets, the two halves
            // of the wave taking alternate sources
            const double dA = anchor_diff(J);
#pragma unroll 1
            for (int rg = 0; rg < RG; ++rg) {
                float t[D];
                const Off *rp = row_off + (row0 + rg * 32 + r32);
#pragma unroll
                for (int k = 0; k < D; ++k) t[k] = static_cast<float>(target_t(dA, rp, k));
#pragma unroll 1
                for (int cs = 0; cs < CH; cs += 2) {
                    const int cj = cs + h;
                    float ss = 0.f;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        // through a scalar: a bit cast whose operand is a vector
                        // element reads the vector's first element in this compiler
                        const unsigned wv = __builtin_bit_cast(uintx4_t, s_a[buf][k / 4][cj])[k % 4];
                        const float dd = t[k] - __builtin_bit_cast(float, wv);
                        ss = __builtin_fmaf(dd, dd, ss);
                    }
                    if constexpr (MAT) {
                        const float sd = __builtin_sqrtf(ss);
                        const float e = __builtin_amdgcn_exp2f(-LOG2E_F * sd);
                        acc[rg] = __builtin_fmaf(__builtin_fmaf(sd, e, e), s_q[buf][cj], acc[rg]);
                    } else {
                        acc[rg] = __builtin_fmaf(__builtin_amdgcn_exp2f(-ss), s_q[buf][cj], acc[rg]);
                    }
                }
            }
        }
        // close a partial-sum group after the last stage of a tile
        if (ci % NCH == NCH - 1 && ((J + 1) % a.gtiles == 0 || J + 1 == J1)) {
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                float sum = acc[rg];
                sum += __shfl_xor(sum, 32, WAVE);
                acc[rg] = 0.f;
                const int64_t i = row0 + rg * 32 + r32;
                if (h == 0) {
                    if (a.ngroups == 1) {
                        if (i < a.n_rows && a.square) sum += static_cast<float>(a.shift) * P::q(q[i]);
                        out[i] = (i < a.n_rows) ? sum : 0.f;
                    } else {
                        out[static_cast<int64_t>(J / a.gtiles) * a.n_pad_rows + i] = sum;
                    }
                }
            }
        }
        if (ci + 1 < C1) stage_store(buf ^ 1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- staged matrix-core exponent
//
// The Gaussian product of k_kmvp_mg (the exponent [2t, c] . [o, 1] on the
// matrix cores; in FP64 with the operand scaled by 256, the table exponential
// and the far clamp) for the large compiled dimensions: FP64 above d = 16,
// FP32 / BF16 above d = 48 (where the split-f16 operands no longer fit).  With
// MAT, the FP64 Matern-3/2 product at every compiled dimension from 2: the
// contraction [o, 1, |o'|^2] . [-2 log2(e)^2 t, |t'|^2, 1] gives
// G = (log2(e) s)^2, and each pair adds 2^(-u) (q + u ln2 q), u = sqrt(G).
// The sources of a column tile pass through LDS 64 (d = 48: 32) at a time
// (double buffered), a wave owns 2 groups of 16
// targets (a block half a row tile), and the target operand is formed per
// column tile by each lane for its own coordinates 4 kc + g only (lane group
// g), with |t|^2 summed over the four lane groups by two exchanges: no lane
// forms or holds all d coordinates.  Wide tiles take the direct form with the
// same coordinate split (each pair's squared distance summed over the lane
// groups; the first group accumulates).
template <int D, int PREC, bool MAT>
__global__ __launch_bounds__(BLOCK) void k_kmvp_mgw(KArgs a) {
    if (a.active != nullptr && *a.active == 0) return;
    using P = Prec<PREC>;
    using M = MG<PREC>;
    using T = typename M::T;
    using V4 = typename M::V4;
    using Off = typename P::Off;
    using Q = typename P::Q;
    constexpr bool TAB = PREC == KRR_FP64;  // table exponential (Gaussian: scaled operand, far clamp)
    // chunks of 4 over the d + 1 coordinates [o, 1] (Matern: d + 2, [o, 1, |o'|^2])
    constexpr int DK = (D + (MAT ? 2 : 1) + 3) / 4;
    constexpr double L2E = 1.4426950408889634074;
    constexpr int RG = 2;             // groups of 16 targets per wave
    constexpr int HB = 2;             // blocks per 256-row tile
    // sources per LDS stage (32 at d = 48: the staging registers then leave
    // room for two waves per SIMD, 29% faster; at d = 64 the smaller stage
    // keeps one wave and measured slower)
    constexpr int CH = D == 48 ? 32 : 64;
    constexpr int NCH = TILE / CH;
    constexpr int LDC = CH + 2;       // padded LDS row
    constexpr int NA = (D * CH + BLOCK - 1) / BLOCK;  // staged offsets per thread
    __shared__ T s_off[2][D][LDC];
    __shared__ __align__(32) T s_q[2][CH];
    // Matern: ln2 q and the source constant |o'|^2 = log2(e)^2 |o|^2
    __shared__ __align__(32) T s_q2[MAT ? 2 : 1][MAT ? CH : 4];
    __shared__ T s_e[MAT ? 2 : 1][MAT ? CH : 1];
    // FP64: the table of 2^(j/256) (exp2_tab; a 2048-entry form with one FMA
    // fewer measured no faster here)
    constexpr int TN = 256;
    __shared__ double s_exp2[TAB ? TN : 1];
    if constexpr (TAB) s_exp2[threadIdx.x] = EXP2_TABLE256[threadIdx.x];
    const Off *__restrict__ off = static_cast<const Off *>(a.off);
    const Off *__restrict__ row_off = static_cast<const Off *>(a.row_off);
    const Q *__restrict__ q = static_cast<const Q *>(a.q);
    const T *__restrict__ qw = static_cast<const T *>(a.qw);
    const int64_t n_pad = a.n_pad;

    const int nrb = a.nrowblocks * HB;
    const int lb = static_cast<int>(blockIdx.x);
    const int bh = lb % nrb, by = lb / nrb;
    const int bx = bh / HB;  // row tile
    const int tid = threadIdx.x;
    const int lane = tid % WAVE;
    const int r16 = lane % 16, g = lane / 16;
    // FP64: A row r16 of a 16-source step holds source (r16 % 4) * 4 + r16 / 4,
    // so that lane l's four accumulator rows are the contiguous sources
    // 4 (l / 16) + v, as they are in FP32 without the permutation
    const int asrc = M::permute_rows ? (r16 % 4) * 4 + r16 / 4 : r16;
    const int64_t row0 = static_cast<int64_t>(bx) * BLOCK + (bh % HB) * (BLOCK / HB) + (tid / WAVE) * (16 * RG);
    T acc[RG];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) acc[rg] = T(0);
    T *__restrict__ out = static_cast<T *>(a.out);

    const int J0 = by * a.tps;
    const int J1 = min(a.ntiles, J0 + a.tps);
    const int C0 = J0 * NCH, C1 = J1 * NCH;
    T st_o[NA], st_q = T(0), st_e = T(0);
    auto stage_load = [&](int ci) {
        const int J = ci / NCH;
        const int64_t j0 = static_cast<int64_t>(J) * TILE + (ci % NCH) * CH;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = u * BLOCK + tid;
            if (D * CH % BLOCK == 0 || e < D * CH) st_o[u] = P::off(off[(e / CH) * n_pad + j0 + e % CH]);
        }
        if (tid < CH) {
            st_q = (MAT || a.tile_r2[J] > P::wide) ? static_cast<T>(P::q(q[j0 + tid])) : qw[j0 + tid];
            if constexpr (MAT && TAB) st_e = static_cast<T>(L2E * L2E * a.sq[j0 + tid]);
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = u * BLOCK + tid;
            if (D * CH % BLOCK == 0 || e < D * CH) s_off[buf][e / CH][e % CH] = st_o[u];
        }
        if (tid < CH) {
            s_q[buf][tid] = st_q;
            if constexpr (MAT) {
                s_q2[buf][tid] = static_cast<T>(0.69314718055994530942) * st_q;  // ln 2 in T's precision
                if constexpr (TAB) s_e[buf][tid] = st_e;
            }
        }
    };
    // this lane's coordinates 4 kc + g of t = x - a_J for target group rg, and
    // the partial |t|^2 over them
    auto target_part = [&](int J, int rg, T (&tv)[DK]) -> double {
        const int64_t i = row0 + rg * 16 + r16;
        double tp = 0.0;
#pragma unroll
        for (int kc = 0; kc < DK; ++kc) {
            const int dim = 4 * kc + g;
            const int dc = min(dim, D - 1);
            const double td = (a.row_anchor[static_cast<int64_t>(bx) * D + dc] - a.anchor[static_cast<int64_t>(J) * D + dc]) +
                              static_cast<double>(P::off(row_off[dc * a.n_pad_rows + i]));
            tv[kc] = dim < D ? static_cast<T>(td) : T(0);
            tp = __builtin_fma(static_cast<double>(tv[kc]), static_cast<double>(tv[kc]), tp);
        }
        return tp;
    };
    auto group_sum = [&](auto v) {
        v += __shfl_xor(v, 16, WAVE);
        return v + __shfl_xor(v, 32, WAVE);
    };

    if (C0 < C1) {
        stage_load(C0);
        stage_store(0);
    }
    __syncthreads();
    T bval[RG][DK];
    for (int ci = C0; ci < C1; ++ci) {
        const int buf = (ci - C0) & 1;
        if (ci + 1 < C1) stage_load(ci + 1);
        const int J = ci / NCH;
        const bool wide = a.tile_r2[J] > P::wide;
        if constexpr (MAT && !TAB) {
            // FP32 / BF16: |o'|^2 of the offsets as staged (rounded), so that the
            // source constant matches the product's offsets
            if (tid < CH) {
                T so = T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) so = M::fma(s_off[buf][k][tid], s_off[buf][k][tid], so);
                s_e[buf][tid] = static_cast<T>(L2E * L2E) * so;
            }
            __syncthreads();
        }
        if (!wide && ci % NCH == 0) {
            const double nj = a.tile_nj[J];
            const double far_t2 = static_cast<double>(a.tile_far64[J]);
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                T tv[DK];
                const double tt = group_sum(target_part(J, rg, tv));
                // FP64: operand scaled by N for exp2_tab; a target whose every
                // exponent against the tile is <= -1100 gets -2000 (exp2 is 0 in
                // FP64 either way), which keeps the scaled exponents in int range
                if constexpr (MAT) {
                    // [-2 log2(e)^2 t, |t'|^2, 1]: the product forms (log2(e) s)^2
#pragma unroll
                    for (int kc = 0; kc < DK; ++kc) {
                        const int dim = 4 * kc + g;
                        bval[rg][kc] = dim < D ? static_cast<T>(-2.0 * L2E * L2E) * tv[kc]
                                               : (dim == D ? static_cast<T>(L2E * L2E * tt) : (dim == D + 1 ? T(1) : T(0)));
                    }
                } else {
                    const bool far = TAB && tt > far_t2;
                    const T sc = TAB ? T(TN) : T(1);
                    const T c = far ? T(-2000.0 * TN) : static_cast<T>(-tt - nj) * sc;
#pragma unroll
                    for (int kc = 0; kc < DK; ++kc) {
                        const int dim = 4 * kc + g;
                        bval[rg][kc] = dim < D ? (far ? T(0) : T(2) * sc * tv[kc]) : (dim == D ? c : T(0));
                    }
                }
            }
        }
        if (!wide) {
#pragma unroll
            for (int st = 0; st < CH / 16; ++st) {
                T av[DK];
#pragma unroll
                for (int kc = 0; kc < DK; ++kc) {
                    const int dim = 4 * kc + g;
                    if (4 * kc + 3 < D) {
                        av[kc] = s_off[buf][dim][st * 16 + asrc];
                    } else {
                        // the last chunks: offsets below d, then the constant 1 (Matern:
                        // then |o'|^2) and zeros
                        const T o = s_off[buf][min(dim, D - 1)][st * 16 + asrc];
                        T v = M::fma(o, static_cast<T>(dim < D), static_cast<T>(dim == D));
                        if constexpr (MAT) v = M::fma(s_e[buf][st * 16 + asrc], static_cast<T>(dim == D + 1), v);
                        av[kc] = v;
                    }
                }
                const V4 qv = *reinterpret_cast<const V4 *>(&s_q[buf][st * 16 + 4 * g]);
                V4 qv2;
                if constexpr (MAT) qv2 = *reinterpret_cast<const V4 *>(&s_q2[buf][st * 16 + 4 * g]);
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    // FP64 at d = 32 and 64: two accumulators over alternate chunks
                    // (half as long a chain of dependent matrix-core operations)
                    // measured 4% faster; at d = 24 and 48 their registers cost the
                    // second wave, and FP32 at d = 64 ran slower with them
                    constexpr bool ACC2 = TAB && (D == 32 || D == 64);
                    V4 G = V4{T(0), T(0), T(0), T(0)}, G1 = G;
#pragma unroll
                    for (int kc = 0; kc < DK; ++kc) {
                        if (ACC2 && (kc & 1))
                            G1 = M::mfma(av[kc], bval[rg][kc], G1);
                        else
                            G = M::mfma(av[kc], bval[rg][kc], G);
                    }
                    if constexpr (ACC2) G += G1;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if constexpr (MAT) {
                            // G = (log2(e) s)^2: (1 + s) e^(-s) q = 2^(-u) (q + u ln2 q), u = sqrt(G)
                            T u, ex;
                            if constexpr (TAB) {
                                u = __builtin_sqrt(__builtin_fabs(G[v]));
                                ex = exp2_tab<TN>(__builtin_fmax(-u * TN, -2000.0 * TN), s_exp2);
                            } else {
                                u = __builtin_amdgcn_sqrtf(__builtin_fabsf(G[v]));
                                ex = __builtin_amdgcn_exp2f(-u);
                            }
                            acc[rg] = M::fma(ex, M::fma(u, qv2[v], qv[v]), acc[rg]);
                        } else if constexpr (TAB) {
                            acc[rg] = M::fma(exp2_tab<TN>(G[v], s_exp2), qv[v], acc[rg]);
                        } else {
                            acc[rg] = M::fma(P::ex2(G[v]), qv[v], acc[rg]);
                        }
                    }
                }
            }
        } else {
            // wide tile: the direct form; each pair's squared distance summed over
            // the lane groups' coordinates, accumulated by the first group
#pragma unroll 1
            for (int rg = 0; rg < RG; ++rg) {
                T tv[DK];
                target_part(J, rg, tv);
#pragma unroll 1
                for (int col = 0; col < CH; ++col) {
                    T sp = T(0);
#pragma unroll
                    for (int kc = 0; kc < DK; ++kc) {
                        const int dim = 4 * kc + g;
                        const T o = s_off[buf][min(dim, D - 1)][col];
                        const T dd = dim < D ? tv[kc] - o : T(0);
                        sp = M::fma(dd, dd, sp);
                    }
                    const T ss = group_sum(sp);
                    T val;
                    if constexpr (MAT) {
                        const T sd = sqrt(ss);
                        const T ex = P::ex2(-static_cast<T>(L2E) * sd);
                        val = M::fma(sd, ex, ex) * s_q[buf][col];
                    } else {
                        val = P::ex2(-ss) * s_q[buf][col];
                    }
                    acc[rg] += g == 0 ? val : T(0);
                }
            }
        }
        // close a partial-sum group after the last stage of a tile
        if (ci % NCH == NCH - 1 && ((J + 1) % a.gtiles == 0 || J + 1 == J1)) {
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                const T sum = group_sum(acc[rg]);
                acc[rg] = T(0);
                const int64_t i = row0 + rg * 16 + r16;
                if (g == 0) {
                    if (a.ngroups == 1) {
                        out[i] = (i < a.n_rows) ? sum + (a.square ? static_cast<T>(a.shift) * P::q(q[i]) : T(0)) : T(0);
                    } else {
                        out[static_cast<int64_t>(J / a.gtiles) * a.n_pad_rows + i] = sum;
                    }
                }
            }
        }
        if (ci + 1 < C1) stage_store(buf ^ 1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- plans and tuning

// Partial-sum groups: the sources are cut into groups of gtiles consecutive
// column tiles (a function of the source count only), each group's sum is
// formed in one block in a fixed order and the groups are added in order, so a
// product's result does not depend on the launch shape the autotuner picks.
int kmvp_group_tiles(const Prepared &C) {
    const int g = C.ntiles / 32;
    return g < 1 ? 1 : (g > 16 ? 16 : g);
}

int kmvp_ngroups(const Prepared &C) {
    const int gt = kmvp_group_tiles(C);
    return (C.ntiles + gt - 1) / gt;
}

// Column splits (blocks per row tile): from 1 to the group count.
int kmvp_max_splits(const Prepared &P) { return kmvp_ngroups(P); }

// The symmetric products (k_kmvp_ms FP64, compiled dimensions up to 16;
// k_kmvp_mhs FP32 / BF16, up to 12, and 16 with groups of 8 tiles or more): Gaussian point sets, groups of gs tiles with gs fixed by the tile count, so
// that the summation order does not depend on tuning: about 100 groups up to
// 1000 tiles, groups of 10 tiles above (clustered sets skip most tile pairs, and
// small groups leave enough blocks with work), and at most about 512 groups
// (the partial sums hold one slot per group and point).
static bool sym_capable(const Prepared &P) {
    return (P.kernel == KRR_KERNEL_GAUSS || P.kernel == KRR_KERNEL_MATERN32) && P.dpad <= 16 &&
           P.ntiles <= 512 * MS_MAX_GROUP_TILES;
}
int kmvp_sym_group_tiles(const Prepared &P) {
    const int a = (P.ntiles + 99) / 100, b = (P.ntiles + 511) / 512;
    const int gs = a < 10 ? a : 10;
    return gs > b ? gs : b;
}
int kmvp_sym_ngroups(const Prepared &P) {
    const int gs = kmvp_sym_group_tiles(P);
    return (P.ntiles + gs - 1) / gs;
}
// Partial-sum slots of a square product's scratch (either layout).
int kmvp_parts_slots(const Prepared &P) {
    const int a = kmvp_ngroups(P), b = sym_capable(P) ? kmvp_sym_ngroups(P) : 0;
    return a > b ? a : b;
}

static KmvpPlan plan_for(const Prepared &P, int splits) {
    KmvpPlan pl;
    const int ng = kmvp_ngroups(P), gt = kmvp_group_tiles(P);
    if (splits < 1) splits = 1;
    if (splits > ng) splits = ng;
    const int gpb = (ng + splits - 1) / splits;  // groups per block
    pl.tiles_per_split = gpb * gt;
    pl.splits = (ng + gpb - 1) / gpb;
    return pl;
}

static KmvpPlan heuristic_plan(const Prepared &P) {
    const int target_blocks = 4096;
    return plan_for(P, (target_blocks + P.ntiles - 1) / P.ntiles);
}

namespace {
struct TuneKey {
    int prec, dpad, ntiles;  // prec: krr_prec + 16 x krr_kernel
    bool operator<(const TuneKey &o) const {
        return prec != o.prec ? prec < o.prec : dpad != o.dpad ? dpad < o.dpad : ntiles < o.ntiles;
    }
};
std::map<TuneKey, int> g_tuned;
std::mutex g_tune_mu;
bool g_tune_loaded = false;

// Optional persistent cache: KRR_TUNE_CACHE names a text file of lines
// "prec dpad ntiles splits".
void tune_cache_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("KRR_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int a, b, c, d;
    while (std::fscanf(f, "%d %d %d %d", &a, &b, &c, &d) == 4) g_tuned[TuneKey{a, b, c}] = d;
    std::fclose(f);
}

void tune_cache_append(const TuneKey &k, int splits) {
    const char *path = std::getenv("KRR_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d\n", k.prec, k.dpad, k.ntiles, splits);
    std::fclose(f);
}
}  // namespace

bool tune_lookup(int key, int dpad, int ntiles, int *value) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tuned.find(TuneKey{key, dpad, ntiles});
    if (it == g_tuned.end()) return false;
    *value = it->second;
    return true;
}

void tune_store(int key, int dpad, int ntiles, int value) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    g_tuned[TuneKey{key, dpad, ntiles}] = value;
    tune_cache_append(TuneKey{key, dpad, ntiles}, value);
}

KmvpPlan kmvp_plan(const Prepared &P, int prec) {
    // KRR_KMVP_SPLITS=k forces k column splits (used to check that results do
    // not depend on the launch shape)
    if (const char *v = std::getenv("KRR_KMVP_SPLITS")) {
        const int k = std::atoi(v);
        if (k > 0) return plan_for(P, k);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tuned.find(TuneKey{prec + 16 * P.kernel, P.dpad, P.ntiles});
    if (it != g_tuned.end()) return plan_for(P, it->second);
    return heuristic_plan(P);
}

size_t kmvp_scratch_bytes(const Prepared &P) {
    const size_t parts = static_cast<size_t>(kmvp_parts_slots(P)) * P.n_pad * 8;
    return align_up(parts, 256) + align_up(static_cast<size_t>(P.n_pad) * 8, 256);
}

KmvpScratch carve_kmvp_scratch(Carver &cv, const Prepared &P) {
    KmvpScratch k;
    k.parts = cv.take<double>(static_cast<size_t>(kmvp_parts_slots(P)) * P.n_pad);
    k.qw = cv.take<double>(P.n_pad);
    return k;
}

// Products up to d = 16 take a matrix-core exponent kernel (split-f16 for FP32
// and BF16, FP64 matrix cores for FP64; Matern: split-f16 for FP32 and BF16),
// the rest the VALU kernels.
// KRR_KMVP_VALU=1 forces the VALU kernel and KRR_KMVP_MG32=1 the FP32
// matrix-core form for FP32 / BF16 (both used to cross-check the kernels).
static bool use_valu_kernel() {
    const char *v = std::getenv("KRR_KMVP_VALU");
    return v && v[0] == '1';
}
// KRR_NO_TILE_SKIP=1 computes far tile pairs too (their terms are exactly zero;
// used to check that skipping them changes nothing)
static bool use_tile_skip() {
    const char *v = std::getenv("KRR_NO_TILE_SKIP");
    return !(v && v[0] == '1');
}
// KRR_KMVP_SYM_SLOTS=1: the symmetric products add their source terms into the
// slots in memory even where a column group fits in LDS (tests compare the two)
static bool sym_slots_in_memory() {
    const char *v = std::getenv("KRR_KMVP_SYM_SLOTS");
    return v && v[0] == '1';
}
static bool use_fp32_matrix_kernel() {
    const char *v = std::getenv("KRR_KMVP_MG32");
    return v && v[0] == '1';
}

template <int D, int PREC>
static hipError_t launch_kmvp(const KArgs &a, int kernel, hipStream_t s) {
    using P = Prec<PREC>;
    if (kernel == KRR_KERNEL_MATERN32) {
        // FP64 at d >= 2 (at d = 1 the VALU form measured faster), FP32 / BF16
        // above d = 48 (below, the split-f16 forms)
        if constexpr ((PREC == KRR_FP64 && D >= 2) || D > 48) {
            if (!use_valu_kernel()) {
                hipLaunchKernelGGL((k_kmvp_mgw<D, PREC, true>), dim3(a.nrowblocks * 2 * a.splits), dim3(BLOCK), 0, s,
                                   a);
                return hipGetLastError();
            }
        }
        if constexpr (D > 16 && D <= 48 && PREC != KRR_FP64) {
            if (!use_valu_kernel()) {
                hipLaunchKernelGGL((k_kmvp_mhw<D, PREC, true>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a);
                return hipGetLastError();
            }
        }
        if constexpr (D <= 16 && PREC != KRR_FP64) {
            if (!use_valu_kernel()) {
                hipLaunchKernelGGL((k_kmvp_mh<D, PREC, true>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a);
                return hipGetLastError();
            }
        }
        if constexpr (D > 16) {
            hipLaunchKernelGGL((k_kmvp_hd<D, PREC, true>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a,
                               static_cast<const typename P::Off *>(a.pm), static_cast<const typename P::T *>(a.qw),
                               a.anchor, static_cast<typename P::T *>(a.out));
        } else {
            hipLaunchKernelGGL((k_kmvp_matern<D, PREC>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a,
                               static_cast<const typename P::Off *>(a.off), static_cast<const typename P::Q *>(a.q),
                               a.anchor, static_cast<typename P::T *>(a.out));
        }
        return hipGetLastError();
    }
    if constexpr (D > 16 && D <= 48 && PREC != KRR_FP64) {
        if (!use_valu_kernel()) {
            hipLaunchKernelGGL((k_kmvp_mhw<D, PREC, false>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a);
            return hipGetLastError();
        }
    }
    if constexpr (D <= 16) {
        if (!use_valu_kernel()) {
            if constexpr (PREC != KRR_FP64) {
                if (!use_fp32_matrix_kernel()) {
                    hipLaunchKernelGGL((k_kmvp_mh<D, PREC, false>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s,
                                       a);
                    return hipGetLastError();
                }
            }
            hipLaunchKernelGGL((k_kmvp_mg<D, PREC>), dim3(a.nrowblocks * (4 / mg_groups<D, PREC>()) * a.splits),
                               dim3(BLOCK), 0, s, a);
            return hipGetLastError();
        }
    }
    if constexpr ((D > 16 && PREC == KRR_FP64) || D > 48) {
        if (!use_valu_kernel()) {
            hipLaunchKernelGGL((k_kmvp_mgw<D, PREC, false>), dim3(a.nrowblocks * 2 * a.splits), dim3(BLOCK), 0, s, a);
            return hipGetLastError();
        }
    }
    if constexpr (D > 16) {
        hipLaunchKernelGGL((k_kmvp_hd<D, PREC, false>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a,
                           static_cast<const typename P::Off *>(a.pm), static_cast<const typename P::T *>(a.qw),
                           a.anchor, static_cast<typename P::T *>(a.out));
    } else {
        hipLaunchKernelGGL((k_kmvp<D, PREC>), dim3(a.nrowblocks * a.splits), dim3(BLOCK), 0, s, a,
                           static_cast<const typename P::Off *>(a.off), static_cast<const typename P::T *>(a.qw),
                           a.anchor, static_cast<typename P::T *>(a.out));
    }
    return hipGetLastError();
}

// KRR_KMVP_SYM=0 keeps the square products one-sided (used to
// cross-check the symmetric kernels); so do KRR_KMVP_VALU=1, KRR_KMVP_MG32=1
// (FP32 / BF16) and KRR_KMVP_SPLITS
static bool use_sym_kernel(const Prepared &P, int prec) {
    if (!sym_capable(P) || use_valu_kernel() || std::getenv("KRR_KMVP_SPLITS")) return false;
    // FP32 / BF16: up to the compiled dimension 12, where it measured faster
    // (N = 1e5: 4-10 % at d = 4-12, 15 % on the kriging shape, 20 % on the
    // clustered one); at 16 only with groups of at least 8 tiles (N above
    // about 180,000: 8 % at N = 2e5), where a row unit meets enough column
    // tiles to repay its set-up (N = 1e5, groups of 4: 11 % slower)
    // Matern-3/2 (FP32 / BF16): at every compiled dimension up to 16, groups of
    // 4 tiles included (its pair costs more: N = 1e5, 1.26-1.41x at d = 3-12,
    // 1.14x at d = 16; N = 2e5, d = 16: 1.24x); FP64: see k_kmvp_ms
    const bool mat = P.kernel == KRR_KERNEL_MATERN32;
    if (prec == KRR_FP64 ? P.dpad > 16
                         : (P.dpad > 16 || (P.dpad == 16 && kmvp_sym_group_tiles(P) < 8 && !mat) ||
                            use_fp32_matrix_kernel()))
        return false;
    const char *v = std::getenv("KRR_KMVP_SYM");
    return !(v && v[0] == '0');
}

template <int D>
static hipError_t launch_kmvp_sym(const KArgs &a, bool mat, hipStream_t s) {
    if constexpr (ms_supported<D>()) {
        const int nb = a.ngroups * (a.ngroups + 1) / 2;
        if (mat)
            hipLaunchKernelGGL((k_kmvp_ms<D, true>), dim3(nb), dim3(BLOCK), 0, s, a);
        else
            hipLaunchKernelGGL((k_kmvp_ms<D, false>), dim3(nb), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <int D, int PREC>
static hipError_t launch_kmvp_sym_h(const KArgs &a, bool mat, hipStream_t s) {
    const int nb = a.ngroups * (a.ngroups + 1) / 2;
    if (mat)
        hipLaunchKernelGGL((k_kmvp_mhs<D, PREC, true>), dim3(nb), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((k_kmvp_mhs<D, PREC, false>), dim3(nb), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_kmvp_sym_hd(int dpad, const KArgs &a, bool mat, hipStream_t s) {
    switch (dpad) {
        case 1: return launch_kmvp_sym_h<1, PREC>(a, mat, s);
        case 2: return launch_kmvp_sym_h<2, PREC>(a, mat, s);
        case 3: return launch_kmvp_sym_h<3, PREC>(a, mat, s);
        case 4: return launch_kmvp_sym_h<4, PREC>(a, mat, s);
        case 6: return launch_kmvp_sym_h<6, PREC>(a, mat, s);
        case 8: return launch_kmvp_sym_h<8, PREC>(a, mat, s);
        case 12: return launch_kmvp_sym_h<12, PREC>(a, mat, s);
        case 16: return launch_kmvp_sym_h<16, PREC>(a, mat, s);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_kmvp_sym_d(int dpad, const KArgs &a, bool mat, hipStream_t s) {
    switch (dpad) {
        case 1: return launch_kmvp_sym<1>(a, mat, s);
        case 2: return launch_kmvp_sym<2>(a, mat, s);
        case 3: return launch_kmvp_sym<3>(a, mat, s);
        case 4: return launch_kmvp_sym<4>(a, mat, s);
        case 6: return launch_kmvp_sym<6>(a, mat, s);
        case 8: return launch_kmvp_sym<8>(a, mat, s);
        case 12: return launch_kmvp_sym<12>(a, mat, s);
        case 16: return launch_kmvp_sym<16>(a, mat, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PREC>
static hipError_t launch_kmvp_d(int dpad, const KArgs &a, int kernel, hipStream_t s) {
    switch (dpad) {
        case 1: return launch_kmvp<1, PREC>(a, kernel, s);
        case 2: return launch_kmvp<2, PREC>(a, kernel, s);
        case 3: return launch_kmvp<3, PREC>(a, kernel, s);
        case 4: return launch_kmvp<4, PREC>(a, kernel, s);
        case 6: return launch_kmvp<6, PREC>(a, kernel, s);
        case 8: return launch_kmvp<8, PREC>(a, kernel, s);
        case 12: return launch_kmvp<12, PREC>(a, kernel, s);
        case 16: return launch_kmvp<16, PREC>(a, kernel, s);
        case 24: return launch_kmvp<24, PREC>(a, kernel, s);
        case 32: return launch_kmvp<32, PREC>(a, kernel, s);
        case 48: return launch_kmvp<48, PREC>(a, kernel, s);
        case 64: return launch_kmvp<64, PREC>(a, kernel, s);
        default: return hipErrorInvalidValue;
    }
}

// The three kernels of one product: prescale, product, partial-sum finish.
// R: targets (rows), C: sources (columns); R == C for the square product.
static hipError_t kmvp_run(const Prepared &R, const Prepared &C, int prec, const KmvpPlan &pl, double shift,
                           const void *q, void *y, const KmvpScratch &sc, const int *active, bool timed_slot,
                           hipStream_t s) {
    const bool square = (&R == &C);
    // the symmetric kernels for square products (plan.sym_gs > 0)
    const bool sym = square && pl.sym_gs > 0;
    KArgs a;
    a.n_rows = R.n;
    a.n_pad_rows = R.n_pad;
    a.nrowblocks = R.ntiles;
    a.row_anchor = R.anchor;
    a.n_pad = C.n_pad;
    a.ntiles = C.ntiles;
    a.splits = pl.splits;
    a.tps = pl.tiles_per_split;
    a.gtiles = sym ? pl.sym_gs : kmvp_group_tiles(C);
    a.ngroups = sym ? (C.ntiles + pl.sym_gs - 1) / pl.sym_gs : kmvp_ngroups(C);
    a.anchor = C.anchor;
    a.tile_r2 = C.tile_r2;
    a.tile_nj = C.tile_nj;
    a.tile_far = C.tile_far;
    a.tile_far64 = C.tile_far64;
    a.sq = C.sq64;
    a.slots = prec == KRR_FP32 ? C.slot32 : prec == KRR_BF16 ? C.slot16 : nullptr;
    a.q = q;
    a.qw = sc.qw;
    a.shift = square ? shift : 0.0;
    a.square = square ? 1 : 0;
    a.active = active;
    a.row_r2 = use_tile_skip() ? R.tile_r2 : nullptr;
    a.zmem = sym_slots_in_memory() ? 1 : 0;
    a.skip_count = nullptr;
    const bool use_parts = a.ngroups > 1 || sym;
    a.out = use_parts ? sc.parts : y;
    const void *w = prec == KRR_FP64 ? static_cast<const void *>(C.w64)
                    : prec == KRR_FP32 ? static_cast<const void *>(C.w32)
                                       : static_cast<const void *>(C.w16);
    a.w = w;
    const dim3 gc((C.n_pad + BLOCK - 1) / BLOCK);
    if (C.kernel == KRR_KERNEL_GAUSS) {  // the Matern product reads q itself
        switch (prec) {
            case KRR_FP64: hipLaunchKernelGGL(k_prescale<KRR_FP64>, gc, dim3(BLOCK), 0, s, C.n_pad, q, w, sc.qw, active); break;
            case KRR_FP32: hipLaunchKernelGGL(k_prescale<KRR_FP32>, gc, dim3(BLOCK), 0, s, C.n_pad, q, w, sc.qw, active); break;
            default: hipLaunchKernelGGL(k_prescale<KRR_BF16>, gc, dim3(BLOCK), 0, s, C.n_pad, q, w, sc.qw, active); break;
        }
        KRR_HIP(hipGetLastError());
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timed =
        timed_slot && profile_slot(prec, static_cast<double>(R.n) * static_cast<double>(C.n), &ev0, &ev1,
                                   static_cast<double>(R.n_pad) * static_cast<double>(C.n_pad), &a.skip_count);
    if (timed) KRR_HIP(hipEventRecord(ev0, s));
    hipError_t e;
    switch (prec) {
        case KRR_FP64:
            a.off = C.off64;
            a.pm = C.pm64;
            a.row_off = R.off64;
            e = sym ? launch_kmvp_sym_d(C.dpad, a, C.kernel == KRR_KERNEL_MATERN32, s)
                    : launch_kmvp_d<KRR_FP64>(C.dpad, a, C.kernel, s);
            break;
        case KRR_FP32:
            a.off = C.off32;
            a.pm = C.pm32;
            a.row_off = R.off32;
            e = sym ? launch_kmvp_sym_hd<KRR_FP32>(C.dpad, a, C.kernel == KRR_KERNEL_MATERN32, s)
                    : launch_kmvp_d<KRR_FP32>(C.dpad, a, C.kernel, s);
            break;
        case KRR_BF16:
            a.off = C.offb;
            a.pm = C.pmb;
            a.row_off = R.offb;
            e = sym ? launch_kmvp_sym_hd<KRR_BF16>(C.dpad, a, C.kernel == KRR_KERNEL_MATERN32, s)
                    : launch_kmvp_d<KRR_BF16>(C.dpad, a, C.kernel, s);
            break;
        default: return hipErrorInvalidValue;
    }
    KRR_HIP(e);
    if (timed) KRR_HIP(hipEventRecord(ev1, s));
    if (use_parts) {
        const int sq = square ? 1 : 0;
        const int ng = a.ngroups;
        auto fgrid = [&](int rows) { return dim3(static_cast<unsigned>((R.n_pad + rows - 1) / rows)); };
        switch (prec) {
            case KRR_FP64:
                hipLaunchKernelGGL(k_kmvp_finish<KRR_FP64>, fgrid(finish_rows<KRR_FP64>()), dim3(BLOCK), 0, s, R.n,
                                   R.n_pad, ng, sc.parts, q, shift, sq, y, active);
                break;
            case KRR_FP32:
                hipLaunchKernelGGL(k_kmvp_finish<KRR_FP32>, fgrid(finish_rows<KRR_FP32>()), dim3(BLOCK), 0, s, R.n,
                                   R.n_pad, ng, sc.parts, q, shift, sq, y, active);
                break;
            default:
                hipLaunchKernelGGL(k_kmvp_finish<KRR_BF16>, fgrid(finish_rows<KRR_BF16>()), dim3(BLOCK), 0, s, R.n,
                                   R.n_pad, ng, sc.parts, q, shift, sq, y, active);
                break;
        }
        KRR_HIP(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t kmvp_sorted(const Prepared &P, int prec, double shift, const void *q, void *y, const KmvpScratch &sc,
                       const int *active, hipStream_t s) {
    KmvpPlan pl;
    if (use_sym_kernel(P, prec))
        pl.sym_gs = kmvp_sym_group_tiles(P);
    else
        pl = kmvp_plan(P, prec);
    return kmvp_run(P, P, prec, pl, shift, q, y, sc, active, true, s);
}

// Rectangular product y = K_hat(targets, sources) q on sorted vectors (targets
// order of T, sources order of S).  Both sets prepared with the same sigma.
hipError_t kmvp_cross_sorted(const Prepared &T, const Prepared &S, int prec, const void *q, void *y,
                             const KmvpScratch &sc, hipStream_t s) {
    const int target_blocks = 4096;
    const KmvpPlan pl = plan_for(S, (target_blocks + T.ntiles - 1) / T.ntiles);
    return kmvp_run(T, S, prec, pl, 0.0, q, y, sc, nullptr, true, s);
}

size_t kmvp_cross_scratch_bytes(const Prepared &T, const Prepared &S) {
    return align_up(static_cast<size_t>(kmvp_max_splits(S)) * T.n_pad * 8, 256) +
           align_up(static_cast<size_t>(S.n_pad) * 8, 256);
}

KmvpScratch carve_kmvp_cross_scratch(Carver &cv, const Prepared &T, const Prepared &S) {
    KmvpScratch k;
    k.parts = cv.take<double>(static_cast<size_t>(kmvp_max_splits(S)) * T.n_pad);
    k.qw = cv.take<double>(S.n_pad);
    return k;
}

// Time every candidate split count on this point set and keep the fastest.
// q must be a valid input vector of the precision; y is overwritten.
hipError_t kmvp_tune(const Prepared &P, int prec, const void *q, void *y, const KmvpScratch &sc, hipStream_t s) {
    // a stream being captured into a graph gets the default shape: timing it
    // would synchronise inside the capture
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (s != nullptr && hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        return hipSuccess;
    if (use_sym_kernel(P, prec)) return hipSuccess;  // its launch shape is fixed
    const TuneKey key{prec + 16 * P.kernel, P.dpad, P.ntiles};  // kernel type in the key
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        if (g_tuned.count(key)) return hipSuccess;
    }
    static const int cands[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    const double pairs = static_cast<double>(P.n_pad) * static_cast<double>(P.n_pad);
    const int reps = pairs > 1e11 ? 1 : 3;
    hipEvent_t e0, e1;
    KRR_HIP(hipEventCreate(&e0));
    KRR_HIP(hipEventCreate(&e1));
    int best = heuristic_plan(P).splits;
    float best_ms = 1e30f;
    int last = -1;
    for (int c : cands) {
        const KmvpPlan pl = plan_for(P, c);
        if (pl.splits == last) continue;
        last = pl.splits;
        hipError_t err = kmvp_run(P, P, prec, pl, 0.0, q, y, sc, nullptr, false, s);
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int r = 0; r < reps && err == hipSuccess; ++r)
            err = kmvp_run(P, P, prec, pl, 0.0, q, y, sc, nullptr, false, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return err;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = pl.splits;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
    tune_cache_append(key, best);
    return hipSuccess;
}

// ---------------------------------------------------------------- launch timing

namespace {
struct ProfileState {
    bool on = false;
    std::vector<hipEvent_t> ev;  // 2 per record
    std::vector<int> prec;
    std::vector<double> pairs, pad_pairs;
    size_t used = 0;
    int64_t dropped = 0;
};
ProfileState g_prof;
}  // namespace

// Row-tile rows x column tiles that the far-tile skipping products left out,
// per product precision, while profiling (one 64-bit counter per precision on
// each device; the kernels add to it through its address).
__device__ unsigned long long g_skipped[3];

static unsigned long long *skip_counter(int prec) {
    static unsigned long long *addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_skipped)) != hipSuccess) return nullptr;
        addr[dev] = static_cast<unsigned long long *>(p);
    }
    return addr[dev] + prec;
}

namespace {
thread_local bool g_prof_suspended = false;
}

void profile_suspend(bool on) { g_prof_suspended = on; }

int progress_every() {
    static const int every = [] {
        const char *v = std::getenv("KRR_PROGRESS");
        const int k = v ? std::atoi(v) : 0;
        return k > 0 ? k : 0;
    }();
    return every;
}

bool profile_slot(int prec, double pairs, hipEvent_t *start, hipEvent_t *stop, double pad_pairs,
                  unsigned long long **skip) {
    if (!g_prof.on || g_prof_suspended) return false;
    if (g_prof.used >= g_prof.prec.size()) {
        ++g_prof.dropped;
        return false;
    }
    const size_t k = g_prof.used++;
    g_prof.prec[k] = prec;
    g_prof.pairs[k] = pairs;
    g_prof.pad_pairs[k] = pad_pairs > 0.0 ? pad_pairs : pairs;
    *start = g_prof.ev[2 * k];
    *stop = g_prof.ev[2 * k + 1];
    if (skip) *skip = skip_counter(prec);
    return true;
}

int profile_begin(int max_launches) {
    if (max_launches < 1) return KRR_EINVAL;
    if (g_prof.on) return KRR_EINVAL;
    const size_t want = static_cast<size_t>(max_launches);
    while (g_prof.ev.size() < 2 * want) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return KRR_EHIP;
        g_prof.ev.push_back(e);
    }
    g_prof.prec.assign(want, 0);
    g_prof.pairs.assign(want, 0.0);
    g_prof.pad_pairs.assign(want, 0.0);
    g_prof.used = 0;
    g_prof.dropped = 0;
    const unsigned long long zero[3] = {0, 0, 0};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_skipped), zero, sizeof(zero), 0, hipMemcpyHostToDevice) != hipSuccess)
        return KRR_EHIP;
    g_prof.on = true;
    return KRR_OK;
}

int profile_end(krr_profile_stats *out) {
    if (!g_prof.on) return KRR_EINVAL;
    g_prof.on = false;
    krr_profile_stats st;
    std::memset(&st, 0, sizeof(st));
    double pad[3] = {0.0, 0.0, 0.0};
    for (size_t k = 0; k < g_prof.used; ++k) {
        if (hipEventSynchronize(g_prof.ev[2 * k + 1]) != hipSuccess) return KRR_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_prof.ev[2 * k], g_prof.ev[2 * k + 1]) != hipSuccess) return KRR_EHIP;
        krr_profile_entry &e = st.prec[g_prof.prec[k]];
        e.launches += 1;
        e.total_ms += ms;
        e.pairs += g_prof.pairs[k];
        pad[g_prof.prec[k]] += g_prof.pad_pairs[k];
    }
    unsigned long long skipped[3] = {0, 0, 0};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpyFromSymbol(skipped, HIP_SYMBOL(g_skipped), sizeof(skipped), 0, hipMemcpyDeviceToHost) != hipSuccess)
        return KRR_EHIP;
    for (int p = 0; p < 3; ++p)
        if (pad[p] > 0.0)  // skipped tile pairs, in the algorithmic (unpadded) pair count
            st.prec[p].pairs_skipped = st.prec[p].pairs * (static_cast<double>(skipped[p]) * TILE / pad[p]);
    st.dropped = g_prof.dropped;
    if (out) *out = st;
    return KRR_OK;
}

}  // namespace krr
