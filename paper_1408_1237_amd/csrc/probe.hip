// Issue-rate probe (measurement support for the product rooflines).
//
// Six register-only kernels, each timed with HIP events on the caller's
// stream, measure on the device at hand:
//   rates[0]  FP32 FMA lane-operations per second (8 independent chains);
//   rates[1]  exp2 + dependent FMA pairs per second (the VALU kernels' inner
//             step: one v_exp_f32 feeding one v_fmac_f32);
//   rates[2]  16x16x4 FP32 matrix-core pairs per second (4 MACs per pair);
//   rates[3]  pairs per second of the matrix-core exponent kernel's mix: per
//             1024 pairs four v_mfma_f32_16x16x4f32, 16 v_exp_f32 and 16 FMAs
//             per lane, the matrix-core results of one step feeding the next
//             step's exponentials;
//   rates[4]  the same for the split-f16 kernel's mix: per 1024 pairs one
//             v_mfma_f32_32x32x16_f16, 16 v_exp_f32 and 16 FMAs per lane;
//   rates[5]  FP64 exp2 (the library's exp2_f64) + dependent FP64 FMA pairs
//             per second (the FP64 products' per-pair VALU work), with one
//             FP64 add per pair that varies the argument.
// Comparing rates[3] with rates[1] and rates[2] shows whether the matrix-core
// and VALU work of one SIMD overlap.  The kernels write one float per thread
// into the workspace (so nothing is dead code); no memory is allocated.
#include <cstdio>

#include "krr_internal.h"

namespace krr {

namespace {

typedef float pf4 __attribute__((ext_vector_type(4)));
typedef float pf16 __attribute__((ext_vector_type(16)));
typedef _Float16 ph8 __attribute__((ext_vector_type(8)));
constexpr int PSTEPS = 256;
constexpr int PBLOCKS = 256 * 16;  // 4096 blocks of 256 threads

__global__ __launch_bounds__(BLOCK) void kp_fma(float *out, float c) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = 0.001f * (k + 1) + gid * 1e-9f;
    for (int i = 0; i < PSTEPS; ++i)
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __builtin_fmaf(v[k], c, 0.5f);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
    out[gid] = s;
}

__global__ __launch_bounds__(BLOCK) void kp_expfma(float *out, float c) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    float a[16], acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = -0.01f * k - gid * 1e-9f;
    for (int i = 0; i < PSTEPS; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k % 4] = __builtin_fmaf(__builtin_amdgcn_exp2f(a[k]), c, acc[k % 4]);
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = a[k] - c * 1e-6f;
    }
    out[gid] = acc[0] + acc[1] + acc[2] + acc[3];
}

__global__ __launch_bounds__(BLOCK) void kp_mfma(float *out, float c) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    const float a = -0.01f * (threadIdx.x % 16);
    float b[4];
    pf4 G[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        b[r] = 0.02f * r + gid * 1e-9f;
        G[r] = pf4{0.f, 0.f, 0.f, 0.f};
    }
    for (int i = 0; i < PSTEPS; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) G[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a * c, b[r], G[r], 0, 0, 0);
    out[gid] = G[0][0] + G[1][1] + G[2][2] + G[3][3];
}

__global__ __launch_bounds__(BLOCK) void kp_mix(float *out, float c) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    float a = -0.01f * (threadIdx.x % 16), b[4], acc[4] = {0.f, 0.f, 0.f, 0.f};
    const pf4 q = {1.f, 0.5f, 0.25f, 0.125f};
    pf4 G[2][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        b[r] = 0.02f * r + gid * 1e-9f;
        G[0][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[r], pf4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    for (int i = 0; i < PSTEPS; i += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float an = a * c + h;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                G[h ^ 1][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(an, b[r], pf4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = __builtin_fmaf(__builtin_amdgcn_exp2f(G[h][r][v]), q[v], acc[r]);
            a = an;
        }
    }
    out[gid] = acc[0] + acc[1] + acc[2] + acc[3];
}

__global__ __launch_bounds__(BLOCK) void kp_mix_h(float *out, float c) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    ph8 a, b;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = static_cast<_Float16>(-0.01f * (threadIdx.x % 16) - 0.001f * i);
        b[i] = static_cast<_Float16>(0.02f + gid * 1e-9f);
    }
    pf16 G[2];
    G[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, pf16{}, 0, 0, 0);
    for (int i = 0; i < PSTEPS; i += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            a[0] = static_cast<_Float16>(static_cast<float>(a[0]) * c + h);
            G[h ^ 1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, pf16{}, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v)
                acc[v % 4] = __builtin_fmaf(__builtin_amdgcn_exp2f(G[h][v]), 0.5f + v, acc[v % 4]);
        }
    }
    out[gid] = acc[0] + acc[1] + acc[2] + acc[3];
}

__global__ __launch_bounds__(BLOCK) void kp_exp64(float *out, float c) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    double a[8], acc[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = -0.37 * k - gid * 1e-9;
    const double cd = c;
    for (int i = 0; i < PSTEPS; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k % 2] = __builtin_fma(exp2_f64(a[k]), cd, acc[k % 2]);
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = a[k] - cd * 1e-6;
    }
    out[gid] = static_cast<float>(acc[0] + acc[1]);
}

}  // namespace

size_t probe_workspace_bytes() { return static_cast<size_t>(PBLOCKS) * BLOCK * sizeof(float); }

hipError_t probe_issue_rates(double *rates, void *ws, hipStream_t s) {
    float *out = static_cast<float *>(ws);
    hipEvent_t e0, e1;
    KRR_HIP(hipEventCreate(&e0));
    KRR_HIP(hipEventCreate(&e1));
    const double threads = static_cast<double>(PBLOCKS) * BLOCK;
    const double waves = threads / WAVE;
    // work per launch: FMA lane-ops, exp2+FMA pairs, matrix-core pairs, the two
    // mixes' pairs, FP64 exp2+FMA pairs
    const double work[6] = {threads * PSTEPS * 8, threads * PSTEPS * 16, waves * PSTEPS * 4 * 256,
                            waves * PSTEPS * 1024, waves * PSTEPS * 1024, threads * PSTEPS * 8};
    hipError_t err = hipSuccess;
    for (int k = 0; k < 6 && err == hipSuccess; ++k) {
        auto launch = [&]() {
            switch (k) {
                case 0: hipLaunchKernelGGL(kp_fma, dim3(PBLOCKS), dim3(BLOCK), 0, s, out, 0.9999f); break;
                case 1: hipLaunchKernelGGL(kp_expfma, dim3(PBLOCKS), dim3(BLOCK), 0, s, out, 1.0001f); break;
                case 2: hipLaunchKernelGGL(kp_mfma, dim3(PBLOCKS), dim3(BLOCK), 0, s, out, 1.0001f); break;
                case 3: hipLaunchKernelGGL(kp_mix, dim3(PBLOCKS), dim3(BLOCK), 0, s, out, 1.0001f); break;
                case 4: hipLaunchKernelGGL(kp_mix_h, dim3(PBLOCKS), dim3(BLOCK), 0, s, out, 1.0001f); break;
                default: hipLaunchKernelGGL(kp_exp64, dim3(PBLOCKS), dim3(BLOCK), 0, s, out, 1.0001f); break;
            }
            return hipGetLastError();
        };
        err = launch();  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int r = 0; r < 5 && err == hipSuccess; ++r) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess) rates[k] = work[k] * 5 / (static_cast<double>(ms) * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err;
}

}  // namespace krr
