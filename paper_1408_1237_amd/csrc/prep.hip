// Point preparation for the kernel products: scaling, Morton ordering, tile
// anchors and per-precision offsets and weights (layout described in
// krr_internal.h).  Runs once per solve; O(N log N) and negligible next to the
// O(N^2) products.
#include <rocprim/device/device_radix_sort.hpp>

#include <cmath>

#include "krr_internal.h"
#include "split16.h"

namespace krr {

static const int kDims[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};

int dim_instance(int d) {
    for (int v : kDims)
        if (v >= d) return v;
    return 0;
}

Prepared carve_prepared(Carver &cv, int64_t n, int d) {
    Prepared P;
    P.n = n;
    P.d = d;
    P.dpad = dim_instance(d);
    P.n_pad = (n + TILE - 1) / TILE * TILE;
    P.ntiles = static_cast<int>(P.n_pad / TILE);
    P.perm = cv.take<int32_t>(P.n_pad);
    P.anchor = cv.take<double>(static_cast<size_t>(P.ntiles) * P.dpad);
    P.tile_r2 = cv.take<double>(P.ntiles);
    P.tile_nj = cv.take<double>(P.ntiles);
    P.tile_far = cv.take<float>(P.ntiles);
    P.tile_far64 = cv.take<float>(P.ntiles);
    P.off64 = cv.take<double>(static_cast<size_t>(P.dpad) * P.n_pad);
    P.off32 = cv.take<float>(static_cast<size_t>(P.dpad) * P.n_pad);
    P.offb = cv.take<float>(static_cast<size_t>(P.dpad) * P.n_pad);
    P.w64 = cv.take<double>(P.n_pad);
    P.w32 = cv.take<float>(P.n_pad);
    P.w16 = cv.take<float>(P.n_pad);
    P.sq64 = cv.take<double>(P.n_pad);
    if (P.dpad > 16) {
        P.pm64 = cv.take<double>(static_cast<size_t>(P.dpad) * P.n_pad);
        P.pm32 = cv.take<float>(static_cast<size_t>(P.dpad) * P.n_pad);
        P.pmb = cv.take<float>(static_cast<size_t>(P.dpad) * P.n_pad);
    }
    const int oct = 2 * split_chunks(P.dpad);
    if (oct > 0) {
        P.slot32 = cv.take<half8_t>(static_cast<size_t>(oct) * P.n_pad);
        P.slot16 = cv.take<half8_t>(static_cast<size_t>(oct) * P.n_pad);
    }
    P.flags = cv.take<int>(4);
    return P;
}

size_t prepared_bytes(int64_t n, int d) {
    Carver cv(nullptr);
    carve_prepared(cv, n, d);
    return cv.off + 256;
}

// keys (2 buffers) + values (2 buffers) + bbox + sort scratch bound
static size_t sort_scratch_bound(int64_t n) { return (size_t(16) << 20) + static_cast<size_t>(n) * 16; }

size_t prep_temp_bytes(int64_t n) {
    Carver cv(nullptr);
    cv.take<uint64_t>(n);
    cv.take<uint64_t>(n);
    cv.take<int32_t>(n);
    cv.take<int32_t>(n);
    cv.take<double>(2 * KRR_MAX_DIM * 1024);
    cv.take<double>(2 * KRR_MAX_DIM);
    cv.take<char>(sort_scratch_bound(n));
    return cv.off + 256;
}

// ---------------------------------------------------------------- reductions

template <typename T, class Op>
__device__ T block_reduce(T v, Op op, T *lds /* >= BLOCK/WAVE */) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off /= 2) v = op(v, __shfl_xor(v, off, WAVE));
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x % WAVE) == 0) lds[w] = v;
    __syncthreads();
    T r = lds[0];
    for (int k = 1; k < static_cast<int>(blockDim.x) / WAVE; ++k) r = op(r, lds[k]);
    __syncthreads();
    return r;
}

struct MinOp { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct MaxOp { __device__ double operator()(double a, double b) const { return fmax(a, b); } };

// ---------------------------------------------------------------- kernels

// Per-block min / max of the scaled coordinate t over a slice of points
// (grid: nblk x d); part[(t * 2 + 0|1) * nblk + blk].  Flags non-finite input.
__global__ __launch_bounds__(BLOCK) void k_bbox_partial(const double *__restrict__ x, int64_t n, int d,
                                                        double scale, double *part, int *flags) {
    __shared__ double lds[BLOCK / WAVE];
    const int t = blockIdx.y;
    const int nblk = gridDim.x;
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)nblk * BLOCK) {
        double v = x[i * d + t];
        if (!isfinite(v)) bad = 1;
        v *= scale;
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    if (bad) atomicOr(flags, 1);
    lo = block_reduce(lo, MinOp(), lds);
    hi = block_reduce(hi, MaxOp(), lds);
    if (threadIdx.x == 0) {
        part[(t * 2 + 0) * nblk + blockIdx.x] = lo;
        part[(t * 2 + 1) * nblk + blockIdx.x] = hi;
    }
}

__global__ void k_bbox_final(const double *part, int nblk, int d, double *bbox) {
    const int t = threadIdx.x;
    if (t >= d) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
        lo = fmin(lo, part[(t * 2 + 0) * nblk + b]);
        hi = fmax(hi, part[(t * 2 + 1) * nblk + b]);
    }
    bbox[2 * t] = lo;
    bbox[2 * t + 1] = hi;
}

// Morton code: the first dm = min(d, 63) scaled coordinates quantised to
// bits = min(63 / dm, 31) bits each over the bounding box, bits interleaved.
__global__ __launch_bounds__(BLOCK) void k_morton(const double *__restrict__ x, int64_t n, int d, double scale,
                                                  const double *__restrict__ bbox, int dm, int bits,
                                                  uint64_t *keys, int32_t *vals) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i >= n) return;
    const double qmax = static_cast<double>((uint64_t(1) << bits) - 1);
    uint64_t code = 0;
    for (int t = 0; t < dm; ++t) {
        const double lo = bbox[2 * t], hi = bbox[2 * t + 1];
        const double ext = hi - lo;
        double f = ext > 0 ? (x[i * d + t] * scale - lo) / ext : 0.0;
        f = fmin(fmax(f, 0.0), 1.0);
        const uint64_t qt = static_cast<uint64_t>(f * qmax);
        for (int b = 0; b < bits; ++b) code |= ((qt >> b) & 1u) << (b * dm + t);
    }
    keys[i] = code;
    vals[i] = static_cast<int32_t>(i);
}

// One block per tile: anchor, offsets, radius, normaliser and weights.
//
// The anchor is the centre of the tile's bounding box, which minimises the
// largest offset, whenever that keeps the tile narrow enough to fold its
// exponent.  A tile too wide to fold anyway (typically a dense group plus a few
// far points that a space-filling order put together) takes the
// coordinate-wise (lower) median instead: it stays inside the group, whose
// offsets then stay short and keep their absolute precision when rounded to
// FP32 or BF16 (with the box centre the group's offsets would be as long as the
// tile, and its pairs' distances would carry that rounding).
__global__ __launch_bounds__(TILE) void k_tiles(const double *__restrict__ x, int64_t n, int d, int dpad,
                                                double scale, const int32_t *__restrict__ sorted_idx,
                                                Prepared P, int matern) {
    __shared__ double lds[TILE / WAVE];
    __shared__ double vals[TILE];
    __shared__ double s_centre[KRR_MAX_DIM];
    __shared__ double s_median[KRR_MAX_DIM];
    const int J = blockIdx.x;
    const int64_t j = static_cast<int64_t>(J) * TILE + threadIdx.x;
    const bool real = j < n;
    const int32_t idx = real ? sorted_idx[j] : -1;
    const int64_t t0 = static_cast<int64_t>(J) * TILE;
    const int nreal = static_cast<int>(n - t0 < TILE ? n - t0 : TILE);  // real points come first in a tile
    P.perm[j] = idx;
    auto coord = [&](int t) { return (real && t < d) ? x[static_cast<int64_t>(idx) * d + t] * scale : 0.0; };
    // pass 1: both candidate anchors, and the radius about the box centre
    double sqc = 0.0;
    for (int t = 0; t < d; ++t) {
        const double v = coord(t);
        const double lo = block_reduce(real ? v : INFINITY, MinOp(), lds);
        const double hi = block_reduce(real ? v : -INFINITY, MaxOp(), lds);
        const double c = 0.5 * (lo + hi);
        // rank of this point's coordinate among the tile's real points (ties by
        // position); the point of rank (nreal - 1) / 2 is the median
        vals[threadIdx.x] = v;
        if (threadIdx.x == 0) {
            s_centre[t] = c;
            s_median[t] = c;  // replaced below (kept only if a non-finite value breaks the ranks)
        }
        __syncthreads();
        if (real) {
            int rank = 0;
            for (int k = 0; k < nreal; ++k) {
                const double u = vals[k];
                rank += (u < v || (u == v && k < static_cast<int>(threadIdx.x))) ? 1 : 0;
            }
            if (rank == (nreal - 1) / 2) s_median[t] = v;
        }
        __syncthreads();  // vals is rewritten for the next coordinate
        const double o = real ? v - c : 0.0;
        sqc += o * o;
    }
    const bool median = block_reduce(sqc, MaxOp(), lds) > WIDE_R2_FP32;
    // pass 2: offsets from the chosen anchor (padding coordinates are zero)
    double sq64 = 0.0, sq32 = 0.0, sq16 = 0.0;
    for (int t = 0; t < dpad; ++t) {
        const double a = t < d ? (median ? s_median[t] : s_centre[t]) : 0.0;
        const double o = real ? coord(t) - a : 0.0;
        const float o32 = static_cast<float>(o);
        if (threadIdx.x == 0) P.anchor[static_cast<size_t>(J) * dpad + t] = a;
        P.off64[t * P.n_pad + j] = o;
        P.off32[t * P.n_pad + j] = o32;
        if (P.pm64 != nullptr) {
            P.pm64[j * dpad + t] = o;
            P.pm32[j * dpad + t] = o32;
        }
        sq64 += o * o;
        sq32 += static_cast<double>(o32) * static_cast<double>(o32);
    }
    // offsets of the BF16 products: rounded to BF16 on a compact tile (this
    // thread reads back the FP32 offsets it wrote)
    const bool compact = block_reduce(sq64, MaxOp(), lds) <= COMPACT_R2_BF16;
    for (int t = 0; t < dpad; ++t) {
        const float o32 = P.off32[t * P.n_pad + j];
        const float ob = compact ? bf16_to_f32(f32_to_bf16_rne(o32)) : o32;
        P.offb[t * P.n_pad + j] = ob;
        if (P.pmb != nullptr) P.pmb[j * dpad + t] = ob;
        sq16 += static_cast<double>(ob) * static_cast<double>(ob);
    }
    const double r2 = block_reduce(fmax(sq64, fmax(sq32, sq16)), MaxOp(), lds);
    const double nj = floor(0.5 * r2);
    if (threadIdx.x == 0) {
        P.tile_r2[J] = r2;
        P.tile_nj[J] = nj;
        // Gaussian: a target at |t| from the anchor has exponent
        // <= -(|t| - R)^2 + R^2 - N_J against every source of the tile, <= -200
        // beyond this |t|^2; Matern: scaled distance >= 111 (exp2 of -log2(e) s
        // is 0 in FP32) beyond (R + 111)^2; 1e-4 margin
        const double u = matern ? sqrt(r2) + 111.0 : sqrt(r2) + sqrt(200.0 + r2 - nj);
        P.tile_far[J] = static_cast<float>(1.0001 * u * u);
        // FP64 Gaussian product: exponents <= -1100 (exp2 is 0 in FP64)
        const double u64 = sqrt(r2) + sqrt(1100.0 + r2 - nj);
        P.tile_far64[J] = static_cast<float>(1.0001 * u64 * u64);
    }
    P.sq64[j] = sq64;
    P.w64[j] = (real && r2 <= WIDE_R2_FP64) ? exp2(nj - sq64) : 0.0;
    P.w32[j] = (real && r2 <= WIDE_R2_FP32) ? static_cast<float>(exp2(nj - sq32)) : 0.0f;
    P.w16[j] = (real && r2 <= WIDE_R2_FP32) ? static_cast<float>(exp2(nj - sq16)) : 0.0f;
}

// Source slot vectors (split16.h) of the FP32 or BF16 offsets, once per set.
// Gaussian: the offsets o and no source constant.  Matern: o' = log2(e) o and
// the constant |o'|^2, so that the product forms (log2(e) r)^2.
template <int D, bool BF, bool MAT>
__global__ __launch_bounds__(BLOCK) void k_slots(Prepared P) {
    const int64_t j = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    if (j >= P.n_pad) return;
    constexpr int KC = split_chunks(D);
    HiLo v[D];
    double so = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float o = BF ? P.offb[k * P.n_pad + j] : P.off32[k * P.n_pad + j];
        if (MAT) {
            o *= LOG2E_F;
            so = __builtin_fma(static_cast<double>(o), static_cast<double>(o), so);
        }
        v[k] = split_f16(o);
    }
    const HiLo one{static_cast<_Float16>(1.f), static_cast<_Float16>(1.f)};
    const HiLo zero{static_cast<_Float16>(0.f), static_cast<_Float16>(0.f)};
    const HiLo e = MAT ? split_f16(static_cast<float>(so)) : zero;
    half8_t *out = static_cast<half8_t *>(BF ? P.slot16 : P.slot32);
#pragma unroll
    for (int w = 0; w < 2 * KC; ++w) out[w * P.n_pad + j] = slot_octet<D, true>(w, v, one, e);
}

template <int D>
static hipError_t launch_slots(const Prepared &P, hipStream_t s) {
    const dim3 g((P.n_pad + BLOCK - 1) / BLOCK);
    if (P.kernel == KRR_KERNEL_MATERN32) {
        hipLaunchKernelGGL((k_slots<D, false, true>), g, dim3(BLOCK), 0, s, P);
        hipLaunchKernelGGL((k_slots<D, true, true>), g, dim3(BLOCK), 0, s, P);
    } else {
        hipLaunchKernelGGL((k_slots<D, false, false>), g, dim3(BLOCK), 0, s, P);
        hipLaunchKernelGGL((k_slots<D, true, false>), g, dim3(BLOCK), 0, s, P);
    }
    return hipGetLastError();
}

static hipError_t build_slots(const Prepared &P, hipStream_t s) {
    switch (P.dpad) {
        case 1: return launch_slots<1>(P, s);
        case 2: return launch_slots<2>(P, s);
        case 3: return launch_slots<3>(P, s);
        case 4: return launch_slots<4>(P, s);
        case 6: return launch_slots<6>(P, s);
        case 8: return launch_slots<8>(P, s);
        case 12: return launch_slots<12>(P, s);
        case 16: return launch_slots<16>(P, s);
        case 24: return launch_slots<24>(P, s);
        case 32: return launch_slots<32>(P, s);
        case 48: return launch_slots<48>(P, s);
        default: return hipSuccess;  // d = 64 takes the VALU kernel
    }
}

__global__ void k_fill_int(int *p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t prepare_points(Prepared &P, const double *x, double sigma, void *temp, size_t temp_bytes,
                          hipStream_t s, int kernel) {
    const int64_t n = P.n;
    const int d = P.d;
    P.kernel = kernel;
    // Gaussian: exp(-r^2 / (2 sigma^2)) = 2^(-||x~_i - x~_j||^2); Matern: the
    // scaled distance ||x~_i - x~_j|| is sqrt(3) r / h
    P.scale = kernel == KRR_KERNEL_MATERN32 ? std::sqrt(3.0) / sigma
                                            : std::sqrt(std::log2(std::exp(1.0))) / (sigma * std::sqrt(2.0));
    Carver cv(temp);
    uint64_t *k0 = cv.take<uint64_t>(n);
    uint64_t *k1 = cv.take<uint64_t>(n);
    int32_t *v0 = cv.take<int32_t>(n);
    int32_t *v1 = cv.take<int32_t>(n);
    double *part = cv.take<double>(2 * KRR_MAX_DIM * 1024);
    double *bbox = cv.take<double>(2 * KRR_MAX_DIM);
    const size_t sort_cap = sort_scratch_bound(n);
    char *sort_tmp = cv.take<char>(sort_cap);
    if (cv.off > temp_bytes) return hipErrorInvalidValue;

    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, P.flags, 4, 0);
    const int nblk = static_cast<int>(std::min<int64_t>(1024, (n + BLOCK - 1) / BLOCK));
    hipLaunchKernelGGL(k_bbox_partial, dim3(nblk, d), dim3(BLOCK), 0, s, x, n, d, P.scale, part, P.flags);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(KRR_MAX_DIM), 0, s, part, nblk, d, bbox);
    const int dm = d < 63 ? d : 63;
    const int bits = (63 / dm) < 31 ? 63 / dm : 31;
    hipLaunchKernelGGL(k_morton, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, x, n, d, P.scale, bbox, dm,
                       bits, k0, v0);
    KRR_HIP(hipGetLastError());
    rocprim::double_buffer<uint64_t> keys(k0, k1);
    rocprim::double_buffer<int32_t> vals(v0, v1);
    size_t need = 0;
    KRR_HIP(rocprim::radix_sort_pairs(nullptr, need, keys, vals, static_cast<size_t>(n), 0u,
                                      static_cast<unsigned>(dm * bits), s));
    if (need > sort_cap) return hipErrorInvalidValue;
    KRR_HIP(rocprim::radix_sort_pairs(sort_tmp, need, keys, vals, static_cast<size_t>(n), 0u,
                                      static_cast<unsigned>(dm * bits), s));
    hipLaunchKernelGGL(k_tiles, dim3(P.ntiles), dim3(TILE), 0, s, x, n, d, P.dpad, P.scale,
                       static_cast<const int32_t *>(vals.current()), P, kernel == KRR_KERNEL_MATERN32 ? 1 : 0);
    KRR_HIP(hipGetLastError());
    return build_slots(P, s);
}

// ---------------------------------------------------------------- gather / scatter

template <typename T>
__device__ inline T cvt(double v);
template <>
__device__ inline double cvt<double>(double v) { return v; }
template <>
__device__ inline float cvt<float>(double v) { return static_cast<float>(v); }

template <typename Tin, typename Tout>
__global__ __launch_bounds__(BLOCK) void k_gather(const int32_t *__restrict__ perm, int64_t n_pad,
                                                  const Tin *__restrict__ src, Tout *__restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i >= n_pad) return;
    const int32_t p = perm[i];
    dst[i] = p >= 0 ? static_cast<Tout>(src[p]) : Tout(0);
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(BLOCK) void k_scatter(const int32_t *__restrict__ perm, int64_t n_pad,
                                                   const Tin *__restrict__ src, Tout *__restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i >= n_pad) return;
    const int32_t p = perm[i];
    if (p >= 0) dst[p] = static_cast<Tout>(src[i]);
}

template <typename Tin, typename Tout>
hipError_t gather_sorted(const Prepared &P, const Tin *src, Tout *dst, hipStream_t s) {
    hipLaunchKernelGGL((k_gather<Tin, Tout>), dim3((P.n_pad + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, P.perm,
                       P.n_pad, src, dst);
    return hipGetLastError();
}
template <typename Tin, typename Tout>
hipError_t scatter_sorted(const Prepared &P, const Tin *src, Tout *dst, hipStream_t s) {
    hipLaunchKernelGGL((k_scatter<Tin, Tout>), dim3((P.n_pad + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, P.perm,
                       P.n_pad, src, dst);
    return hipGetLastError();
}

template hipError_t gather_sorted<double, double>(const Prepared &, const double *, double *, hipStream_t);
template hipError_t gather_sorted<float, float>(const Prepared &, const float *, float *, hipStream_t);
template hipError_t gather_sorted<double, float>(const Prepared &, const double *, float *, hipStream_t);
template hipError_t scatter_sorted<double, double>(const Prepared &, const double *, double *, hipStream_t);
template hipError_t scatter_sorted<float, float>(const Prepared &, const float *, float *, hipStream_t);
template hipError_t scatter_sorted<float, double>(const Prepared &, const float *, double *, hipStream_t);
template hipError_t gather_sorted<float, double>(const Prepared &, const float *, double *, hipStream_t);
template hipError_t scatter_sorted<double, float>(const Prepared &, const double *, float *, hipStream_t);

__global__ __launch_bounds__(BLOCK) void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst,
                                                   int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i < n) dst[i] = f32_to_bf16_rne(src[i]);
}

hipError_t to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace krr
