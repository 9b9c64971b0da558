// Several right-hand sides at once: Y = K_hat Q + shift Q on the matrix cores.
//
// Per pair the kernel value is formed once on the VALU (the folded, tile-
// anchored exponent of krr_internal.h: d fused multiply-adds and one exp2) and
// applied to 16 right-hand sides by one MFMA: with v_mfma_{f32,f64}_16x16x4
// the A operand is a 16 (rows) x 4 (columns) block of K_hat, one value per lane
// (lane l: row l % 16, column l / 16), the B operand the 4 x 16 block of the
// prescaled sources Q'[j][r] = Q[j][r] w_j (lane l: column l / 16, right-hand
// side l % 16), and the 16 x 16 accumulator holds the block of Y (right-hand
// side l % 16; rows 4 (l / 16) + v for FP32, l / 16 + 4 v for FP64, v < 4).
// A wave owns 64 rows (four 16-row blocks, four accumulators) and sweeps the
// columns of its split 4 at a time; a block of 4 waves owns one 256-row tile.
// Partial sums per split are added in fixed order by the finish kernel.
#include <cstdlib>

#include "krr_internal.h"
#include "split16.h"

namespace krr {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct MP;
template <>
struct MP<KRR_FP64> {
    using T = double;
    using Off = double;
    using Acc = doublex4;
    static constexpr double wide = WIDE_R2_FP64;
    static __device__ __forceinline__ T off(Off v) { return v; }
    static __device__ __forceinline__ T ex2(T a) { return exp2_f64(a); }
    static __device__ __forceinline__ T fma(T a, T b, T c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ Acc mfma(T a, T b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct MP<KRR_FP32> {
    using T = float;
    using Off = float;
    using Acc = floatx4;
    static constexpr double wide = WIDE_R2_FP32;
    static __device__ __forceinline__ T off(Off v) { return v; }
    static __device__ __forceinline__ T ex2(T a) { return __builtin_amdgcn_exp2f(a); }
    static __device__ __forceinline__ T fma(T a, T b, T c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ Acc mfma(T a, T b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct MP<KRR_BF16> : MP<KRR_FP32> {
    using Off = float;  // FP32 values, BF16-rounded on compact tiles (prep)
    static __device__ __forceinline__ float off(Off v) { return v; }
};

}  // namespace krr
#include "kmvp_multi.h"
namespace krr {

// 16-row blocks processed together by one wave (register budget); a wave
// covers its 64 rows in 4 / RB passes over the columns.  FP64 keeps 2 RB D
// doubles of target offsets live (oi and t): from D = 6 it takes two row
// blocks, and its column steps are not unrolled, for two waves per SIMD
// instead of one (FP64 16-RHS products 5-7 % faster at d = 6, 8).
template <int D, int PREC>
constexpr int multi_rb() {
    return (PREC == KRR_FP64 ? 4 : 1) * D <= 16 ? 4 : (PREC == KRR_FP64 ? 2 : 1) * D <= 32 ? 2 : 1;
}

// Global-address-space view of a pointer (the batched kernel reads its
// arguments from device memory, where the compiler cannot infer the space).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gp(const void *p) {
    return (const __attribute__((address_space(1))) T *)p;
}

// Columns staged per LDS chunk: the two buffers of offsets and 16 prescaled
// right-hand sides stay within about 40 KB, so several blocks share a CU.
template <int D, int PREC>
constexpr int multi_chunk() {
    constexpr int bytes = (D + 16) * (PREC == KRR_FP64 ? 8 : 4);
    constexpr int fit = 20480 / bytes;
    return fit >= 256 ? 256 : fit >= 128 ? 128 : fit >= 64 ? 64 : 32;
}

template <int D, int PREC>
__device__ __forceinline__ void multi_body(const MArgs &a, int bx, int by, int rbk) {
    using P = MP<PREC>;
    using T = typename P::T;
    using Off = typename P::Off;
    using Acc = typename P::Acc;
    constexpr int RB = multi_rb<D, PREC>();
    constexpr int SC = multi_chunk<D, PREC>();
    constexpr int CPT = TILE / SC;  // chunks per column tile
    constexpr int LDO = SC + 16;
    constexpr int UN = D > 16 ? 1 : (PREC == KRR_FP64 && D >= 6) ? 1 : 4;  // unroll of the column steps (registers)
    // The sources of the current column chunk (offsets and the 16 prescaled
    // right-hand sides) are staged in LDS, double-buffered: the block loads
    // chunk c + 1 from memory while it computes chunk c.
    __shared__ T s_off[2][D][LDO];
    __shared__ __align__(16) T s_b[2][SC][16];
    const auto off = gp<Off>(a.off);
    const auto qb = gp<T>(a.qwt) + static_cast<int64_t>(rbk) * a.n_pad * 16;
    const auto anchor = gp<double>(a.anchor);
    const auto tile_r2 = gp<double>(a.tile_r2);
    const auto tile_nj = gp<double>(a.tile_nj);
    const int64_t n_pad = a.n_pad;
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const int lane = tid % WAVE;
    const int r16 = lane % 16, g = lane / 16;
    T *parts = static_cast<T *>(a.parts) + (static_cast<int64_t>(by) * a.nrb + rbk) * n_pad * 16;
    const int C0 = by * a.tps * CPT;
    const int C1 = min(a.ntiles, (by + 1) * a.tps) * CPT;

    double aI[D];
#pragma unroll
    for (int k = 0; k < D; ++k) aI[k] = anchor[static_cast<int64_t>(bx) * D + k];

    // staging: thread tid loads (source, coordinate / right-hand side) entries
    // of the chunk; SC * (D + 16) entries over the 256 threads
    constexpr int NO = (SC * D + BLOCK - 1) / BLOCK;   // offsets per thread
    constexpr int NB = (SC * 16 + BLOCK - 1) / BLOCK;  // rhs values per thread
    T st_o[NO], st_b[NB];
    auto stage_load = [&](int cidx) {
        const int64_t j0 = static_cast<int64_t>(cidx) * SC;
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int e = u * BLOCK + tid;  // e = k * SC + col
            const int k = e / SC, col = e % SC;
            st_o[u] = (e < SC * D) ? P::off(off[k * n_pad + j0 + col]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = u * BLOCK + tid;  // e = col * 16 + r
            st_b[u] = qb[j0 * 16 + e];
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int e = u * BLOCK + tid;
            if (e < SC * D) s_off[buf][e / SC][e % SC] = st_o[u];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = u * BLOCK + tid;
            s_b[buf][e / 16][e % 16] = st_b[u];
        }
    };

    for (int pass = 0; pass < 4 / RB; ++pass) {
        const int64_t row0 = static_cast<int64_t>(bx) * BLOCK + wave * 64 + pass * RB * 16;
        T oi[RB][D];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int k = 0; k < D; ++k) oi[rb][k] = P::off(off[k * n_pad + row0 + rb * 16 + r16]);
        Acc acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = Acc{0, 0, 0, 0};

        if (C0 < C1) {
            stage_load(C0);
            stage_store(0);
        }
        __syncthreads();
        for (int ci = C0; ci < C1; ++ci) {
            const int buf = (ci - C0) & 1;
            if (ci + 1 < C1) stage_load(ci + 1);
            const int J = ci / CPT;
            const double r2 = tile_r2[J];
            const double nj = tile_nj[J];
            T t[RB][D];
            T c[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                double tt = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double td =
                        (aI[k] - anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(oi[rb][k]);
                    t[rb][k] = static_cast<T>(td);
                    const double tk = static_cast<double>(t[rb][k]);
                    tt = __builtin_fma(tk, tk, tt);
                }
                c[rb] = static_cast<T>(-tt - nj);
            }
            if (r2 <= P::wide) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int k = 0; k < D; ++k) t[rb][k] = t[rb][k] + t[rb][k];
#pragma unroll UN
                for (int st = 0; st < SC; st += 4) {
                    const int cj = st + g;
                    T oc[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) oc[k] = s_off[buf][k][cj];
                    const T b = s_b[buf][cj][r16];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        T arg = P::fma(t[rb][0], oc[0], c[rb]);
#pragma unroll
                        for (int k = 1; k < D; ++k) arg = P::fma(t[rb][k], oc[k], arg);
                        acc[rb] = P::mfma(P::ex2(arg), b, acc[rb]);
                    }
                }
            } else {
#pragma unroll 1
                for (int st = 0; st < SC; st += 4) {
                    const int cj = st + g;
                    T oc[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) oc[k] = s_off[buf][k][cj];
                    const T b = s_b[buf][cj][r16];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        T ss = T(0);
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const T dd = t[rb][k] - oc[k];
                            ss = P::fma(dd, dd, ss);
                        }
                        acc[rb] = P::mfma(P::ex2(-ss), b, acc[rb]);
                    }
                }
            }
            if (ci + 1 < C1) stage_store(buf ^ 1);
            __syncthreads();
        }
        // accumulator layout: FP32 lane l holds rows 4 (l / 16) + v; FP64 lane l
        // holds rows l / 16 + 4 v (right-hand side l % 16 in both)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = (PREC == KRR_FP64) ? g + 4 * v : 4 * g + v;
                parts[(row0 + rb * 16 + rr) * 16 + r16] = acc[rb][v];
            }
    }
}

// ---------------------------------------------------------------- split-f16 exponent
//
// FP32 / BF16 at d <= 16: the kernel values come from the matrix cores too.
// One v_mfma_f32_16x16x32_f16 per 32 slots of the split exponent (split16.h:
// sources as A, the lane's target as B) forms the exponents of 16 sources x 16
// targets; its accumulator gives lane l target l % 16 against sources
// 4 (l / 16) + v (v < 4), which after exp2 is exactly the A operand of the
// 16 x 4 x 16 FP32 product with Q' when its v-th operation takes sources
// v, 4 + v, 8 + v, 12 + v of the step (B reads the Q' rows in that order), so
// no value moves between lanes.  Per 16 sources x 16 targets: one f16 operation
// per 32 slots, 4 exp2 per lane and 4 FP32 operations for 16 right-hand sides.
// Targets far from a tile get the exponent -2000 (as in the single product);
// wide tiles stage plain FP32 offsets in the octet words and take the direct
// form for the kernel values.
template <int D>
constexpr int multi_chunk_h() {
    constexpr int bytes = 2 * split_chunks(D) * 16 + 64;
    constexpr int fit = 20480 / bytes;
    return fit >= 256 ? 256 : fit >= 128 ? 128 : fit >= 64 ? 64 : 32;
}

// Transpose across the four 16-lane rows of a wave: on entry lane row g holds
// o[j] = item (g, j); on exit it holds o[j] = item (j, g).  Two exchange steps
// per 32-bit word: v_permlane32_swap trades the upper lane half of its first
// operand with the lower half of its second (registers j, j + 2), then
// v_permlane16_swap the odd 16-lane rows of its first operand with the even
// rows of its second (registers 2i, 2i + 1).
__device__ __forceinline__ void transpose_rows(half8_t (&o)[4]) {
    uintx4_t R[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) R[j] = __builtin_bit_cast(uintx4_t, o[j]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const unsigned x = R[j][e], y = R[j + 2][e];
            const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
            R[j][e] = r[0];
            R[j + 2][e] = r[1];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const unsigned x = R[2 * i][e], y = R[2 * i + 1][e];
            const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
            R[2 * i][e] = r[0];
            R[2 * i + 1][e] = r[1];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = __builtin_bit_cast(half8_t, R[j]);
}

template <int D, int PREC>
__device__ __forceinline__ void multi_body_h(const MArgs &a, int bx, int by, int rbk) {
    using P = MP<PREC>;
    using Off = typename P::Off;
    constexpr int NOCT = 2 * split_chunks(D);  // prepared octets per source
    constexpr int KC = (NOCT + 3) / 4;         // 32-slot chunks
    constexpr int RB = D <= 8 ? 4 : 2;         // 16-row blocks per pass (register budget)
    constexpr int SC = multi_chunk_h<D>();
    constexpr int CPT = TILE / SC;
    __shared__ __align__(16) half8_t s_a[2][NOCT][SC];
    __shared__ __align__(16) float s_b[2][SC][16];
    const auto off = gp<Off>(a.off);
    const auto slots = gp<half8_t>(a.slots);
    const auto qb = gp<float>(a.qwt) + static_cast<int64_t>(rbk) * a.n_pad * 16;
    const auto anchor = gp<double>(a.anchor);
    const auto tile_r2 = gp<double>(a.tile_r2);
    const auto tile_nj = gp<double>(a.tile_nj);
    const auto tile_far = gp<float>(a.tile_far);
    const int64_t n_pad = a.n_pad;
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const int lane = tid % WAVE;
    const int r16 = lane % 16, g = lane / 16;
    float *parts = static_cast<float *>(a.parts) + (static_cast<int64_t>(by) * a.nrb + rbk) * n_pad * 16;
    const int C0 = by * a.tps * CPT;
    const int C1 = min(a.ntiles, (by + 1) * a.tps) * CPT;
    const half8_t zero8 = __builtin_bit_cast(half8_t, uintx4_t{0u, 0u, 0u, 0u});

    double aI[D];
#pragma unroll
    for (int k = 0; k < D; ++k) aI[k] = anchor[static_cast<int64_t>(bx) * D + k];

    // staging: entry e = w * SC + col (octet w of source col), then the 16 Q'
    // values of each source; on wide tiles octet w holds FP32 offsets 4w .. 4w + 3
    constexpr int NA = (SC * NOCT + BLOCK - 1) / BLOCK;
    constexpr int NB = (SC * 16 + BLOCK - 1) / BLOCK;
    half8_t st_a[NA];
    float st_b[NB];
    auto stage_load = [&](int cidx) {
        const int64_t j0 = static_cast<int64_t>(cidx) * SC;
        const bool wide = tile_r2[cidx / CPT] > P::wide;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = u * BLOCK + tid;
            const int w = e / SC, col = e % SC;
            if (e >= SC * NOCT) {
                st_a[u] = zero8;
            } else if (wide) {
                uintx4_t v;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float o = (4 * w + i < D) ? P::off(off[(4 * w + i) * n_pad + j0 + col]) : 0.f;
                    v[i] = __builtin_bit_cast(unsigned, o);
                }
                st_a[u] = __builtin_bit_cast(half8_t, v);
            } else {
                st_a[u] = slots[w * n_pad + j0 + col];
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) st_b[u] = qb[j0 * 16 + u * BLOCK + tid];
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = u * BLOCK + tid;
            if (e < SC * NOCT) s_a[buf][e / SC][e % SC] = st_a[u];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = u * BLOCK + tid;
            s_b[buf][e / 16][e % 16] = st_b[u];
        }
    };

    for (int pass = 0; pass < 4 / RB; ++pass) {
        const int64_t row0 = static_cast<int64_t>(bx) * BLOCK + wave * 64 + pass * RB * 16;
        // RB = 4: lane l forms the operand of its own target row0 + l (group l / 16)
        // and the four lane rows trade octets (transpose_rows); RB = 2: every lane
        // forms the operands of both of its groups
        constexpr bool XPOSE = RB == 4;
        float oi[XPOSE ? 1 : RB][D];
        if constexpr (XPOSE) {
#pragma unroll
            for (int k = 0; k < D; ++k) oi[0][k] = P::off(off[k * n_pad + row0 + lane]);
        } else {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int k = 0; k < D; ++k) oi[rb][k] = P::off(off[k * n_pad + row0 + rb * 16 + r16]);
        }
        floatx4 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};

        if (C0 < C1) {
            stage_load(C0);
            stage_store(0);
        }
        __syncthreads();
        // the target operand depends on the column tile only: with RB = 4 formed
        // at the tile's first chunk and kept over its CPT chunks (with RB = 2,
        // where registers are short, formed again per chunk)
        half8_t bval[RB][KC];
        for (int ci = C0; ci < C1; ++ci) {
            const int buf = (ci - C0) & 1;
            if (ci + 1 < C1) stage_load(ci + 1);
            const int J = ci / CPT;
            const double r2 = tile_r2[J];
            if (r2 <= P::wide) {
                const float njf = static_cast<float>(tile_nj[J]);
                const float far_t2 = tile_far[J];
#pragma unroll
                for (int rb = 0; rb < (XPOSE ? 1 : RB); ++rb) {
                    if (XPOSE && ci % CPT != 0) break;
                    float t[D];
                    double tt = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double td =
                            (aI[k] - anchor[static_cast<int64_t>(J) * D + k]) + static_cast<double>(oi[rb][k]);
                        t[k] = static_cast<float>(td);
                        tt = __builtin_fma(td, td, tt);
                    }
                    const bool far = static_cast<float>(tt) > far_t2;
                    const _Float16 z16 = static_cast<_Float16>(0.f);
                    HiLo v[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) v[k] = split_f16(far ? 0.f : 2.f * t[k]);
                    const HiLo c = far ? HiLo{static_cast<_Float16>(-2000.f), z16}
                                       : split_f16(-static_cast<float>(tt) - njf);
                    const HiLo c2{z16, z16};
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) {
                        // octet 4 kc + g of the target vector (lane group g)
                        half8_t o[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) o[j] = slot_octet<D, false>(4 * kc + j, v, c, c2);
                        if constexpr (XPOSE) {
                            transpose_rows(o);
#pragma unroll
                            for (int j = 0; j < 4; ++j) bval[j][kc] = o[j];
                        } else {
                            bval[rb][kc] = g == 0 ? o[0] : g == 1 ? o[1] : g == 2 ? o[2] : o[3];
                        }
                    }
                }
#pragma unroll 2
                for (int st = 0; st < SC; st += 16) {
                    half8_t av[KC];
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) {
                        const int w = 4 * kc + g;
                        av[kc] = (w < NOCT) ? s_a[buf][w < NOCT ? w : 0][st + r16] : zero8;
                    }
                    float bq[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) bq[v] = s_b[buf][st + 4 * g + v][r16];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        floatx4 G = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc)
                            G = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[kc], bval[rb][kc], G, 0, 0, 0);
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_amdgcn_exp2f(G[v]), bq[v],
                                                                          acc[rb], 0, 0, 0);
                    }
                }
            } else {
                float t[RB][D];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        float o;
                        if constexpr (XPOSE)
                            o = P::off(off[k * n_pad + row0 + rb * 16 + r16]);
                        else
                            o = oi[rb][k];
                        t[rb][k] = static_cast<float>((aI[k] - anchor[static_cast<int64_t>(J) * D + k]) +
                                                      static_cast<double>(o));
                    }
#pragma unroll 1
                for (int st = 0; st < SC; st += 16) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int cj = st + 4 * g + v;
                        float oc[D];
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            // through a scalar: a bit cast whose operand is a vector
                            // element reads the vector's first element in this compiler
                            const unsigned wv = __builtin_bit_cast(uintx4_t, s_a[buf][k / 4][cj])[k % 4];
                            oc[k] = __builtin_bit_cast(float, wv);
                        }
                        const float b = s_b[buf][cj][r16];
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            float ss = 0.f;
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                const float dd = t[rb][k] - oc[k];
                                ss = __builtin_fmaf(dd, dd, ss);
                            }
                            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_amdgcn_exp2f(-ss), b, acc[rb],
                                                                          0, 0, 0);
                        }
                    }
                }
            }
            if (ci + 1 < C1) stage_store(buf ^ 1);
            __syncthreads();
        }
        // accumulator: lane l holds right-hand side l % 16 of rows 4 (l / 16) + v
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) parts[(row0 + rb * 16 + 4 * g + v) * 16 + r16] = acc[rb][v];
    }
}

// H: the split-f16 exponent body (FP32 / BF16, d <= 16), else the VALU one.
template <int D, int PREC, bool H>
__device__ __forceinline__ void multi_select(const MArgs &a, int bx, int by, int rbk) {
    if constexpr (H && PREC != KRR_FP64 && D <= 16)
        multi_body_h<D, PREC>(a, bx, by, rbk);
    else
        multi_body<D, PREC>(a, bx, by, rbk);
}

// Which body a launch takes: the split-f16 exponent for FP32 / BF16 up to
// d = 16 unless KRR_KMVP_MULTI_VALU=1 (used to cross-check the two).
static bool multi_use_h(int dpad, int prec) {
    const char *v = std::getenv("KRR_KMVP_MULTI_VALU");
    return prec != KRR_FP64 && dpad <= 16 && !(v && v[0] == '1');
}

template <int D, int PREC, bool H>
__global__ __launch_bounds__(BLOCK) void k_kmvp_multi(MArgs a) {
    const int lb = static_cast<int>(blockIdx.x);
    const int bx = lb % a.nrowblocks;
    const int rest = lb / a.nrowblocks;
    multi_select<D, PREC, H>(a, bx, rest % a.splits, rest / a.splits);
}


// Batched over many systems of one dimension: block b runs work item b
// (system, row tile, column chunk, RHS block) with that system's arguments.
__device__ __forceinline__ bool gate_live(const ColGate &g, int c) {
    return (g.a == nullptr || g.a[c] != 0) && (g.b == nullptr || g.b[c] != 0);
}

template <int D, int PREC, bool H>
__global__ __launch_bounds__(BLOCK) void k_kmvp_multi_batched(const MSysB *__restrict__ sys,
                                                              const MItem *__restrict__ items, ColGate gate) {
    const MItem it = items[blockIdx.x];
    const MSysB &m = sys[it.sys];
    if (gate.a != nullptr || gate.b != nullptr) {
        const int live = threadIdx.x < 16 ? gate_live(gate, m.col0 + it.rbk * 16 + threadIdx.x) : 0;
        if (!__syncthreads_or(live)) return;  // block-uniform
    }
    multi_select<D, PREC, H>(m.a, it.bx, it.by, it.rbk);
}

// Q'[rbk][j][r % 16] = Q[p_j + r ldq] * weff_j for r < nrhs (0 beyond), where
// p_j is the original index of sorted position j (perm == nullptr: p_j = j),
// weff_j = w_j on folded tiles and 1 on wide tiles.  BF16: Q rounded first.
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_multi_prescale(int64_t n_pad, int nrhs, int nrb, const int32_t *perm,
                                                          const void *Q_, int64_t ldq, const void *w_,
                                                          const double *tile_r2, void *qwt_) {
    using T = typename MP<PREC>::T;
    const T *Q = static_cast<const T *>(Q_);
    const T *w = static_cast<const T *>(w_);
    T *qwt = static_cast<T *>(qwt_);
    const int64_t idx = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    const int64_t total = n_pad * 16 * nrb;
    if (idx >= total) return;
    const int r16 = static_cast<int>(idx % 16);
    const int64_t j = (idx / 16) % n_pad;
    const int rbk = static_cast<int>(idx / (16 * n_pad));
    const int r = rbk * 16 + r16;
    const int64_t p = perm ? static_cast<int64_t>(perm[j]) : j;
    T v = T(0);
    if (r < nrhs && p >= 0) {
        v = Q[p + static_cast<int64_t>(r) * ldq];
        if (PREC == KRR_BF16) v = bf16_to_f32(f32_to_bf16_rne(static_cast<float>(v)));
        const bool wide = tile_r2[j / TILE] > MP<PREC>::wide;
        v = wide ? v : v * w[j];
    }
    qwt[idx] = v;
}

// Y[p_i + r ldy] = sum_s parts[s][r / 16][i][r % 16] + shift Q[p_i + r ldq], i < n.
// A block takes 64 sorted rows x the 16 right-hand sides of block blockIdx.y, as
// k_multi_finish_b: reads along the [row][16] layout (splits added from the
// first, in order), an LDS turn-over, one wave per column on the way out.
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_multi_finish(int64_t n, int64_t n_pad, int nrhs, int nrb, int splits,
                                                        const int32_t *perm, const void *parts_, const void *Q_,
                                                        int64_t ldq, double shift, void *Y_, int64_t ldy) {
    using T = typename MP<PREC>::T;
    constexpr int ROWS = 64;
    constexpr int PER = ROWS * 16 / BLOCK;
    __shared__ T s_y[16][ROWS + 1];
    const T *parts = static_cast<const T *>(parts_);
    const T *Q = static_cast<const T *>(Q_);
    T *Y = static_cast<T *>(Y_);
    const int rbk = blockIdx.y;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * ROWS;
    if (row0 >= n_pad) return;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int l = threadIdx.x + e * BLOCK;  // row l / 16, right-hand side l % 16
        T acc = T(0);
        for (int k = 0; k < splits; ++k) acc += parts[((static_cast<int64_t>(k) * nrb + rbk) * n_pad + row0) * 16 + l];
        s_y[l % 16][l / 16] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int l = threadIdx.x + e * BLOCK;
        const int c = l / ROWS, il = l % ROWS;
        const int r = rbk * 16 + c;
        if (r >= nrhs) continue;
        const int64_t i = row0 + il;
        const int64_t p = perm ? static_cast<int64_t>(perm[i]) : (i < n ? i : -1);
        if (p < 0) {
            if (!perm) Y[i + static_cast<int64_t>(r) * ldy] = T(0);  // keep sorted vectors zero-padded
            continue;
        }
        T qv = Q[p + static_cast<int64_t>(r) * ldq];
        if (PREC == KRR_BF16) qv = bf16_to_f32(f32_to_bf16_rne(static_cast<float>(qv)));
        Y[p + static_cast<int64_t>(r) * ldy] = s_y[c][il] + static_cast<T>(shift) * qv;
    }
}

// ---------------------------------------------------------------- batched over systems

// Prescale / finish for every system of a batched product (grid.y = system).
// Vectors are the concatenated sorted blocks: system k's column r is at
// base_k + r n_pad_k.
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_multi_prescale_b(const MSysB *__restrict__ S, const void *Qall_,
                                                            int nrhs, ColGate gate) {
    using T = typename MP<PREC>::T;
    const MSysB &m = S[blockIdx.y];
    const int64_t n_pad = m.a.n_pad;
    const int nrb = m.a.nrb;
    const int64_t idx = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (idx >= n_pad * 16 * nrb) return;
    const T *Q = static_cast<const T *>(Qall_) + m.base;
    const T *w = static_cast<const T *>(m.w);
    T *qwt = static_cast<T *>(const_cast<void *>(m.a.qwt));
    const int r16 = static_cast<int>(idx % 16);
    const int64_t j = (idx / 16) % n_pad;
    const int r = static_cast<int>(idx / (16 * n_pad)) * 16 + r16;
    if (!gate_live(gate, m.col0 + r)) return;
    T v = T(0);
    if (r < nrhs) {
        v = Q[j + static_cast<int64_t>(r) * n_pad];
        if (PREC == KRR_BF16) v = bf16_to_f32(f32_to_bf16_rne(static_cast<float>(v)));
        const bool wide = m.a.tile_r2[j / TILE] > MP<PREC>::wide;
        v = wide ? v : v * w[j];
    }
    qwt[idx] = v;
}

// Y = sum over the column chunks of the partial sums + shift Q, per system and
// live column.  A block takes 64 rows x the 16 right-hand sides of one block:
// it reads the [row][16] partial sums along memory (the chunks added from the
// first, in order), turns the 64 x 16 sums over in LDS and writes each column's
// 64 rows with one wave.
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_multi_finish_b(const MSysB *__restrict__ S, const void *Qall_, void *Yall_,
                                                          int nrhs, int inner, ColGate gate) {
    using T = typename MP<PREC>::T;
    constexpr int ROWS = 64;
    constexpr int PER = ROWS * 16 / BLOCK;
    __shared__ T s_y[16][ROWS + 1];
    const MSysB &m = S[blockIdx.y];
    const int64_t n_pad = m.a.n_pad;
    const int nchunk = static_cast<int>(n_pad / ROWS);
    const int nrb = m.a.nrb;
    if (static_cast<int>(blockIdx.x) >= nchunk * nrb) return;
    const int rbk = blockIdx.x / nchunk;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x % nchunk) * ROWS;
    bool any = false;
    for (int c = 0; c < 16; ++c) {
        const int r = rbk * 16 + c;
        any = any || (r < nrhs && gate_live(gate, m.col0 + r));
    }
    if (!any) return;
    const T *parts = static_cast<const T *>(m.a.parts);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int l = threadIdx.x + e * BLOCK;  // row l / 16, right-hand side l % 16
        T acc = T(0);
        for (int k = 0; k < m.a.splits; ++k)
            acc += parts[((static_cast<int64_t>(k) * nrb + rbk) * n_pad + row0) * 16 + l];
        s_y[l % 16][l / 16] = acc;
    }
    __syncthreads();
    T *Y = static_cast<T *>(Yall_) + m.base;
    const T *Q = static_cast<const T *>(Qall_) + m.base;
    const T shift = static_cast<T>(inner ? m.shift_in : m.shift_out);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int l = threadIdx.x + e * BLOCK;
        const int c = l / ROWS, il = l % ROWS;
        const int r = rbk * 16 + c;
        if (r >= nrhs || !gate_live(gate, m.col0 + r)) continue;
        const int64_t i = row0 + il, idx = static_cast<int64_t>(r) * n_pad + i;
        if (i >= m.a.n) {
            Y[idx] = T(0);
            continue;
        }
        T qv = Q[idx];
        if (PREC == KRR_BF16) qv = bf16_to_f32(f32_to_bf16_rne(static_cast<float>(qv)));
        Y[idx] = s_y[c][il] + shift * qv;
    }
}

size_t batched_product_scratch_bytes(const Prepared &P, int nrhs, int min_tps) {
    const int nrb = (nrhs + 15) / 16;
    const int splits = (P.ntiles + min_tps - 1) / min_tps;
    return align_up(static_cast<size_t>(splits) * nrb * P.n_pad * 16 * 8, 256) +
           align_up(static_cast<size_t>(nrb) * P.n_pad * 16 * 8, 256);
}

void fill_msys(MSysB &m, const Prepared &P, int prec, int nrhs, void *scratch, int64_t base, double shift_in,
               double shift_out, int tps) {
    Carver cv(scratch);
    const int nrb = (nrhs + 15) / 16;
    MArgs &a = m.a;
    a.n = P.n;
    a.n_pad = P.n_pad;
    a.ntiles = P.ntiles;
    a.nrowblocks = P.ntiles;
    a.tps = P.ntiles < tps ? P.ntiles : tps;
    a.splits = (P.ntiles + a.tps - 1) / a.tps;
    a.nrb = nrb;
    a.anchor = P.anchor;
    a.tile_r2 = P.tile_r2;
    a.tile_nj = P.tile_nj;
    a.tile_far = P.tile_far;
    a.slots = prec == KRR_FP32 ? P.slot32 : prec == KRR_BF16 ? P.slot16 : nullptr;
    a.parts = cv.take<double>(static_cast<size_t>(a.splits) * nrb * P.n_pad * 16);
    a.qwt = cv.take<double>(static_cast<size_t>(nrb) * P.n_pad * 16);
    a.off = prec == KRR_FP64 ? static_cast<const void *>(P.off64)
            : prec == KRR_FP32 ? static_cast<const void *>(P.off32)
                               : static_cast<const void *>(P.offb);
    m.w = prec == KRR_FP64 ? static_cast<const void *>(P.w64)
          : prec == KRR_FP32 ? static_cast<const void *>(P.w32)
                             : static_cast<const void *>(P.w16);
    m.base = base;
    m.shift_in = shift_in;
    m.shift_out = shift_out;
    m.col0 = 0;
}

template <int D, int PREC>
static hipError_t launch_multi_b(const MSysB *S, const MItem *items, int nitems, ColGate gate, hipStream_t s) {
    if (multi_use_h(D, PREC))
        hipLaunchKernelGGL((k_kmvp_multi_batched<D, PREC, true>), dim3(nitems), dim3(BLOCK), 0, s, S, items, gate);
    else
        hipLaunchKernelGGL((k_kmvp_multi_batched<D, PREC, false>), dim3(nitems), dim3(BLOCK), 0, s, S, items, gate);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_multi_b_d(int dpad, const MSysB *S, const MItem *items, int nitems, ColGate gate,
                                   hipStream_t s) {
    switch (dpad) {
        case 1: return launch_multi_b<1, PREC>(S, items, nitems, gate, s);
        case 2: return launch_multi_b<2, PREC>(S, items, nitems, gate, s);
        case 3: return launch_multi_b<3, PREC>(S, items, nitems, gate, s);
        case 4: return launch_multi_b<4, PREC>(S, items, nitems, gate, s);
        case 6: return launch_multi_b<6, PREC>(S, items, nitems, gate, s);
        case 8: return launch_multi_b<8, PREC>(S, items, nitems, gate, s);
        case 12: return launch_multi_b<12, PREC>(S, items, nitems, gate, s);
        case 16: return launch_multi_b<16, PREC>(S, items, nitems, gate, s);
        case 24: return launch_multi_b<24, PREC>(S, items, nitems, gate, s);
        case 32: return launch_multi_b<32, PREC>(S, items, nitems, gate, s);
        case 48: return launch_multi_b<48, PREC>(S, items, nitems, gate, s);
        case 64: return launch_multi_b<64, PREC>(S, items, nitems, gate, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PREC>
static hipError_t batched_run(const BatchedProduct &bp, const void *Qall, void *Yall, int inner, ColGate gate,
                              hipStream_t s) {
    const dim3 g((bp.max_elems + BLOCK - 1) / BLOCK, bp.nsys);
    hipLaunchKernelGGL(k_multi_prescale_b<PREC>, g, dim3(BLOCK), 0, s, bp.d_sys, Qall, bp.nrhs, gate);
    KRR_HIP(hipGetLastError());
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timed = profile_slot(PREC, bp.pairs * bp.nrhs, &ev0, &ev1);
    if (timed) KRR_HIP(hipEventRecord(ev0, s));
    KRR_HIP(launch_multi_b_d<PREC>(bp.dpad, bp.d_sys, bp.d_items, bp.nitems, gate, s));
    if (timed) KRR_HIP(hipEventRecord(ev1, s));
    const dim3 gf((bp.max_elems + 64 * 16 - 1) / (64 * 16), bp.nsys);
    hipLaunchKernelGGL(k_multi_finish_b<PREC>, gf, dim3(BLOCK), 0, s, bp.d_sys, Qall, Yall, bp.nrhs, inner, gate);
    return hipGetLastError();
}

hipError_t batched_product(const BatchedProduct &bp, const void *Qall, void *Yall, int inner, ColGate gate,
                           hipStream_t s) {
    switch (bp.prec) {
        case KRR_FP64: return batched_run<KRR_FP64>(bp, Qall, Yall, inner, gate, s);
        case KRR_FP32: return batched_run<KRR_FP32>(bp, Qall, Yall, inner, gate, s);
        case KRR_BF16: return batched_run<KRR_BF16>(bp, Qall, Yall, inner, gate, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- host

static int multi_splits(const Prepared &P, int nrb) {
    const int target_blocks = 2048;
    int blocks = P.ntiles * nrb;
    int s = (target_blocks + blocks - 1) / blocks;
    int mx = P.ntiles / 2 > 1 ? P.ntiles / 2 : 1;
    if (mx > 16) mx = 16;
    if (s > mx) s = mx;
    return s < 1 ? 1 : s;
}

size_t kmvp_multi_scratch_bytes(const Prepared &P, int nrhs) {
    const int nrb = (nrhs + 15) / 16;
    const int mx = P.ntiles / 2 > 1 ? (P.ntiles / 2 < 16 ? P.ntiles / 2 : 16) : 1;
    return align_up(static_cast<size_t>(mx) * nrb * P.n_pad * 16 * 8, 256) +
           align_up(static_cast<size_t>(nrb) * P.n_pad * 16 * 8, 256);
}

template <int D, int PREC>
static hipError_t launch_multi(const MArgs &a, hipStream_t s) {
    const dim3 grid(a.nrowblocks * a.splits * a.nrb);
    if (multi_use_h(D, PREC))
        hipLaunchKernelGGL((k_kmvp_multi<D, PREC, true>), grid, dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((k_kmvp_multi<D, PREC, false>), grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_multi_d(int dpad, const MArgs &a, hipStream_t s) {
    switch (dpad) {
        case 1: return launch_multi<1, PREC>(a, s);
        case 2: return launch_multi<2, PREC>(a, s);
        case 3: return launch_multi<3, PREC>(a, s);
        case 4: return launch_multi<4, PREC>(a, s);
        case 6: return launch_multi<6, PREC>(a, s);
        case 8: return launch_multi<8, PREC>(a, s);
        case 12: return launch_multi<12, PREC>(a, s);
        case 16: return launch_multi<16, PREC>(a, s);
        case 24: return launch_multi<24, PREC>(a, s);
        case 32: return launch_multi<32, PREC>(a, s);
        case 48: return launch_multi<48, PREC>(a, s);
        case 64: return launch_multi<64, PREC>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PREC>
static hipError_t multi_run(const Prepared &P, int nrhs, double shift, const int32_t *perm, const void *Q,
                            int64_t ldq, void *Y, int64_t ldy, void *scratch, hipStream_t s) {
    const int nrb = (nrhs + 15) / 16;
    const int splits_req = multi_splits(P, nrb);
    MArgs a;
    a.n = P.n;
    a.n_pad = P.n_pad;
    a.ntiles = P.ntiles;
    a.nrowblocks = P.ntiles;
    a.tps = (P.ntiles + splits_req - 1) / splits_req;
    a.splits = (P.ntiles + a.tps - 1) / a.tps;
    a.nrb = nrb;
    a.anchor = P.anchor;
    a.tile_r2 = P.tile_r2;
    a.tile_nj = P.tile_nj;
    a.tile_far = P.tile_far;
    a.slots = PREC == KRR_FP32 ? P.slot32 : PREC == KRR_BF16 ? P.slot16 : nullptr;
    Carver cv(scratch);
    const int mx = P.ntiles / 2 > 1 ? (P.ntiles / 2 < 16 ? P.ntiles / 2 : 16) : 1;
    a.parts = cv.take<double>(static_cast<size_t>(mx) * nrb * P.n_pad * 16);
    void *qwt = cv.take<double>(static_cast<size_t>(nrb) * P.n_pad * 16);
    a.qwt = qwt;
    const void *w = PREC == KRR_FP64 ? static_cast<const void *>(P.w64)
                    : PREC == KRR_FP32 ? static_cast<const void *>(P.w32)
                                       : static_cast<const void *>(P.w16);
    a.off = PREC == KRR_FP64 ? static_cast<const void *>(P.off64)
            : PREC == KRR_FP32 ? static_cast<const void *>(P.off32)
                               : static_cast<const void *>(P.offb);
    const int64_t tot_pre = P.n_pad * 16 * nrb;
    hipLaunchKernelGGL(k_multi_prescale<PREC>, dim3((tot_pre + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, P.n_pad, nrhs,
                       nrb, perm, Q, ldq, w, P.tile_r2, qwt);
    KRR_HIP(hipGetLastError());
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timed = profile_slot(PREC, static_cast<double>(P.n) * static_cast<double>(P.n) * nrhs, &ev0, &ev1);
    if (timed) KRR_HIP(hipEventRecord(ev0, s));
    KRR_HIP(launch_multi_d<PREC>(P.dpad, a, s));
    if (timed) KRR_HIP(hipEventRecord(ev1, s));
    hipLaunchKernelGGL(k_multi_finish<PREC>, dim3(static_cast<unsigned>((P.n_pad + 63) / 64), nrb), dim3(BLOCK), 0, s,
                       P.n, P.n_pad, nrhs, nrb, a.splits, perm, a.parts, Q, ldq, shift, Y, ldy);
    return hipGetLastError();
}

hipError_t kmvp_multi(const Prepared &P, int prec, int nrhs, double shift, const int32_t *perm, const void *Q,
                      int64_t ldq, void *Y, int64_t ldy, void *scratch, hipStream_t s) {
    switch (prec) {
        case KRR_FP64: return multi_run<KRR_FP64>(P, nrhs, shift, perm, Q, ldq, Y, ldy, scratch, s);
        case KRR_FP32: return multi_run<KRR_FP32>(P, nrhs, shift, perm, Q, ldq, Y, ldy, scratch, s);
        case KRR_BF16: return multi_run<KRR_BF16>(P, nrhs, shift, perm, Q, ldq, Y, ldy, scratch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace krr
