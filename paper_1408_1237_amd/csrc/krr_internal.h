// Internal declarations of the gfx950 kernel-system solver library.
//
// Layout of a prepared point set (all device memory, carved from the caller's
// workspace):
//  * coordinates are pre-scaled by c = sqrt(log2 e) / (sigma sqrt 2), so the
//    Gaussian of eq. (Gaussian) becomes k_ij = 2^(-||xs_i - xs_j||^2);
//  * points are sorted along a Morton (Z-order) curve and grouped in tiles of
//    TILE consecutive points; each tile J has an FP64 anchor a_J (centre of its
//    bounding box) and every point stores its offset o_j = xs_j - a_J in the
//    working precision (FP64, FP32 or bfloat16), structure-of-arrays;
//  * per tile: R2_J = max_j ||o_j||^2 and a normaliser N_J = floor(R2_J / 2);
//    per point and precision: w_j = 2^(N_J - ||o_j||^2) (o_j as rounded in that
//    precision), 0 for padding points.
// With t = x_i - a_J the exponent splits as
//   -||t - o_j||^2 = (2 t . o_j - ||t||^2 - N_J) + (N_J - ||o_j||^2),
// so the inner loop of a product evaluates 2^(c_i + sum_k T_ik o_jk) * (w_j q_j)
// with per-row constants T = 2t, c = -||t||^2 - N_J: d fused multiply-adds, one
// exp2 and one accumulate per pair.  Tiles whose radius exceeds the precision's
// limit use the direct form 2^(-||t - o_j||^2) instead.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/krr.h"
#include "exp2_table.h"

namespace krr {

constexpr int TILE = 256;       // points per anchor tile; also rows per product block
constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int VEC_BLOCKS = 512; // blocks of the vector (reduction) kernels

// Above these squared tile radii (scaled units) a tile uses the direct form.
// The folded exponent adds terms of size up to about 2 R^2, so its absolute
// error grows with R^2: the FP32 / BF16 matrix-core form splits its operands to
// 2^-22 (split16.h), which at R^2 = 40 leaves per-pair exponent errors of at
// most about 2e-5 on the pairs that matter.
constexpr double WIDE_R2_FP32 = 40.0;
constexpr double WIDE_R2_FP64 = 512.0;
// BF16 products round a tile's offsets to BF16 only on compact tiles: BF16
// keeps 8 significant bits, so an offset of length up to R moves by up to
// 2^-8 R, and a pair at scaled distance r changes its exponent by up to
// 2 r 2^-8 R.  At R^2 <= 1 (R <= 1) that is at most about 0.5% of the kernel
// value for the pairs within one scaled unit, which dominate the sums (beside
// BF16's own rounding of q, 2^-8 per entry); tiles of larger radius keep the
// FP32 offsets.
constexpr double COMPACT_R2_BF16 = 1.0;

// 2^a in FP64 for a <= 1023 (device).  a = n + f with n = rint(a) and
// |f| <= 1/2 (the subtraction is exact); 2^f by a near-minimax polynomial of
// degree 10 (Chebyshev fit, coefficients from exp2_coeffs.py; relative error
// about 3e-16 before rounding of the evaluation), scaled by 2^n.  Arguments
// below -1100 are clamped (the result then underflows to 0).
__device__ __forceinline__ double exp2_f64(double a) {
    a = fmax(a, -1100.0);
    const double n = __builtin_rint(a);
    const double f = a - n;
    double p = 7.072585949269223e-09;
    p = __builtin_fma(p, f, 1.0208690299958306e-07);
    p = __builtin_fma(p, f, 1.321544258792169e-06);
    p = __builtin_fma(p, f, 1.5252657260200837e-05);
    p = __builtin_fma(p, f, 0.0001540353044173605);
    p = __builtin_fma(p, f, 0.0013333558230164974);
    p = __builtin_fma(p, f, 0.009618129107606888);
    p = __builtin_fma(p, f, 0.05550410866444772);
    p = __builtin_fma(p, f, 0.24022650695910097);
    p = __builtin_fma(p, f, 0.69314718055995);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_amdgcn_ldexp(p, static_cast<int>(n));
}

// 2^(x / N) for the FP64 products (x = N times the exponent, N = 256 or 4096):
// with n = rint(x), j = n mod N, f = x - n (exact, |f| <= 1/2),
// 2^(x/N) = 2^((n - j)/N) 2^(j/N) 2^(f/N), the middle factor from the correctly
// rounded table in LDS, the last a polynomial of degree 4 (N = 256) or 2
// (N = 4096; relative errors 2e-18 and 2.5e-14, exp2_table.py).  x must lie in
// int range (the caller clamps far targets); 11 or 9 FP64 instructions against
// 15 for exp2_f64.
template <int N>
__device__ __forceinline__ double exp2_tab(double x, const double *__restrict__ tab) {
    static_assert(N == 256 || N == 4096, "table sizes of exp2_table.h");
    constexpr int SH = N == 256 ? 8 : 12;
    const double n = __builtin_rint(x);
    const double f = x - n;
    const int i = static_cast<int>(n);
    double p;
    if constexpr (N == 256) {
        p = EXP2_POLY256[0];
#pragma unroll
        for (int k = 1; k < 5; ++k) p = __builtin_fma(p, f, EXP2_POLY256[k]);
    } else {
        p = EXP2_POLY4096[0];
#pragma unroll
        for (int k = 1; k < 3; ++k) p = __builtin_fma(p, f, EXP2_POLY4096[k]);
    }
    return __builtin_amdgcn_ldexp(p * tab[i & (N - 1)], i >> SH);
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Device counters and scratch for the last-block reductions of one solver.
struct RedScratch {
    unsigned *counters;  // NCOUNTERS
    double *partials;    // VEC_BLOCKS * NPARTIAL_SLOTS doubles (also used as float)
    static constexpr int NCOUNTERS = 16;
    static constexpr int NPARTIAL_SLOTS = 4;
};

struct Prepared {
    int64_t n = 0, n_pad = 0;
    int d = 0, dpad = 0;      // dpad: dimension of the kernel instance (>= d, extra coords 0)
    int ntiles = 0;
    double scale = 0.0;
    int32_t *perm = nullptr;  // n_pad: sorted position -> original index, -1 for padding
    double *anchor = nullptr; // ntiles * dpad
    double *tile_r2 = nullptr;
    double *tile_nj = nullptr;
    float *tile_far = nullptr; // |t|^2 beyond which every exponent against the tile is <= -200
    float *tile_far64 = nullptr; // the same for exponents <= -1100 (FP64 Gaussian product)
    double *off64 = nullptr;  // dpad * n_pad
    float *off32 = nullptr;
    float *offb = nullptr;    // offsets of BF16 products: BF16-rounded on compact tiles (COMPACT_R2_BF16), else FP32
    double *w64 = nullptr;    // n_pad
    float *w32 = nullptr;
    float *w16 = nullptr;
    double *sq64 = nullptr;   // n_pad: ||o_j||^2 (FP64 offsets)
    // point-major copies of the offsets ([n_pad][dpad]) for dpad > 16: the d
    // coordinates of a source are contiguous, so the large-d VALU product
    // reads a group of sources with scalar loads from one base address
    double *pm64 = nullptr;
    float *pm32 = nullptr;
    float *pmb = nullptr;
    // split-f16 source slot vectors of the FP32 and BF16 offsets (split16.h):
    // 2 split_chunks(dpad) octets per point, octet-major ([octet][n_pad]), for dpad <= 48
    void *slot32 = nullptr;
    void *slot16 = nullptr;
    int *flags = nullptr;     // [0]: non-finite input seen
    int kernel = KRR_KERNEL_GAUSS;  // krr_kernel of the products on this set
};

// Sizes of a prepared set.
int dim_instance(int d);  // smallest compiled kernel dimension >= d, 0 if none
size_t prepared_bytes(int64_t n, int d);
size_t prep_temp_bytes(int64_t n);
// Carve a Prepared from the workspace (pointers only).
Prepared carve_prepared(Carver &cv, int64_t n, int d);

// Build the prepared layout from FP64 row-major points; temp is scratch of
// prep_temp_bytes(n).  Returns a HIP error code.
// sigma: the Gaussian bandwidth, or the Matern length scale h (kernel ==
// KRR_KERNEL_MATERN32: coordinates scaled by sqrt(3) / h).
hipError_t prepare_points(Prepared &P, const double *x, double sigma, void *temp, size_t temp_bytes,
                          hipStream_t s, int kernel = KRR_KERNEL_GAUSS);

// Gather an original-order vector into sorted order (padding 0), and back.
template <typename Tin, typename Tout>
hipError_t gather_sorted(const Prepared &P, const Tin *src, Tout *dst, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t scatter_sorted(const Prepared &P, const Tin *src, Tout *dst, hipStream_t s);

// Kernel products on sorted, zero-padded vectors of length n_pad.
// prec: KRR_FP64 (q, y double), KRR_FP32 (float), KRR_BF16 (q: bf16 bits, y float).
struct KmvpPlan {
    int splits = 1;          // column splits
    int tiles_per_split = 0;
    int sym_gs = 0;          // > 0: the symmetric FP64 kernel with groups of sym_gs tiles
};
// Scratch of one product: group partial sums (kmvp_parts_slots x n_pad, 8
// bytes each)
// and the prescaled sources q_j w_j (n_pad, 8 bytes each).
struct KmvpScratch {
    void *parts = nullptr;
    void *qw = nullptr;
};
int kmvp_max_splits(const Prepared &P);
int kmvp_parts_slots(const Prepared &P);
KmvpPlan kmvp_plan(const Prepared &P, int prec);  // tuned, else a heuristic
size_t kmvp_scratch_bytes(const Prepared &P);
KmvpScratch carve_kmvp_scratch(Carver &cv, const Prepared &P);
// y = K_hat q + shift q on sorted vectors.  active: optional device flag; when it
// reads 0 the kernels return at once.
hipError_t kmvp_sorted(const Prepared &P, int prec, double shift, const void *q, void *y, const KmvpScratch &sc,
                       const int *active, hipStream_t s);
// Rectangular product y = K_hat(targets T, sources S) q (sorted orders of T and S).
hipError_t kmvp_cross_sorted(const Prepared &T, const Prepared &S, int prec, const void *q, void *y,
                             const KmvpScratch &sc, hipStream_t s);
size_t kmvp_cross_scratch_bytes(const Prepared &T, const Prepared &S);
KmvpScratch carve_kmvp_cross_scratch(Carver &cv, const Prepared &T, const Prepared &S);
// Several right-hand sides on the matrix cores: Y[p_i + r ldy] = (K_hat Q)_i,r +
// shift Q[p_i + r ldq] with p_i = perm[i] (original order; perm == nullptr: the
// vectors are in sorted order, zero-padded, and Y's padding is zeroed).
// scratch: kmvp_multi_scratch_bytes(P, nrhs).
size_t kmvp_multi_scratch_bytes(const Prepared &P, int nrhs);
hipError_t kmvp_multi(const Prepared &P, int prec, int nrhs, double shift, const int32_t *perm, const void *Q,
                      int64_t ldq, void *Y, int64_t ldy, void *scratch, hipStream_t s);
// Gradient pass (grad.hip): gx (n x d, original order), g_logsigma, g_loggamma
// (device scalars) of -lam^T (dK/dtheta) w.  scratch: grad_scratch_bytes(P).
size_t grad_scratch_bytes(const Prepared &P);
hipError_t kmvp_grad_run(const Prepared &P, int prec, double sigma, double gamma, const double *lam,
                         const double *w, double *gx, double *g_ls, double *g_lg, void *scratch, hipStream_t s);
// Autotuner: time the candidate column splits for (prec, d, N) on this point
// set once per process (and KRR_TUNE_CACHE file) and keep the fastest.
hipError_t kmvp_tune(const Prepared &P, int prec, const void *q, void *y, const KmvpScratch &sc, hipStream_t s);
// The autotuner's cache (in-process, and the KRR_TUNE_CACHE file): an integer
// per (key, dpad, ntiles); single products use key = prec + 16 x kernel, the
// batched products 64 + prec (ntiles: the class's tiles x RHS blocks).
bool tune_lookup(int key, int dpad, int ntiles, int *value);
void tune_store(int key, int dpad, int ntiles, int value);

// Device-resident scalars of one CG solve (T = float for the inner
// preconditioner solve, double for the plain solver).
template <typename T>
struct CgScalars {
    T rr;       // r . r
    T rr0;      // ||rhs||^2 at start
    T thresh;   // stop when rr <= thresh (tol^2 rr0)
    T alpha, beta, pAp;
    int active;     // 1 while iterating
    int iters;      // iterations done
    int maxit;
    int status;     // 0 ok, KRR_BREAKDOWN
    int candidate;  // plain solver: recursive residual reached the tolerance
    int pad_[3];
};

// Device-resident state of one FGMRES solve (FP64), m = restart length.
struct FgmresScalars {
    double bnorm;   // ||b||
    double beta;    // ||r0|| of the current cycle
    double est;     // |g_{j+1}| / ||b||
    double wnorm0;  // ||K z_j|| before orthogonalisation
    int breakdown;  // h_{j+1,j} negligible: happy breakdown
    int nonfinite;
    int pad_[2];
};

// Launch timing (krr_profile_begin / krr_profile_end): when enabled, returns
// the event pair to record around one product kernel of `pairs` pair
// evaluations in precision prec, or false when disabled / the pool is full.
// pad_pairs: the padded pair count of the launch; skip (optional): receives the
// device counter the far-tile skipping kernels add their skipped rows x tiles to.
bool profile_slot(int prec, double pairs, hipEvent_t *start, hipEvent_t *stop, double pad_pairs = 0.0,
                  unsigned long long **skip = nullptr);
int profile_begin(int max_launches);
void profile_suspend(bool on);  // while on, profile_slot hands out no events
int profile_end(krr_profile_stats *out);

// Issue-rate probe (probe.hip): FMA lane-ops/s, exp2+FMA pairs/s, matrix-core
// pairs/s, matrix-core exponent mix pairs/s.  ws: probe_workspace_bytes().
size_t probe_workspace_bytes();
hipError_t probe_issue_rates(double *rates, void *ws, hipStream_t s);

// GPR prediction (predict.hip): the n x 16 block of kernel columns of test
// points j0..j0+15 and the variance reduction 1 - k_j^T W_j.
size_t predict_var_bytes(int64_t n);  // the block and its solution
hipError_t predict_kernel_block(const double *x, int64_t n, int d, const double *xs, int64_t m, int64_t j0,
                                double sigma, int kernel, double *B, hipStream_t s);
hipError_t predict_var_block(const double *B, const double *W, int64_t n, int64_t m, int64_t j0, double *var,
                             hipStream_t s);

// Progress lines on stderr: KRR_PROGRESS=k prints one line every k outer steps
// of a solve (0 or unset: silent).
int progress_every();

// bf16 conversion of a float vector (round to nearest even).
hipError_t to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t s);

__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    uint32_t u = static_cast<uint32_t>(h) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

#define KRR_HIP(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return e_;                \
    } while (0)

}  // namespace krr
