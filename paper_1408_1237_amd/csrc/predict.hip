// GPR prediction (section 2.1): posterior mean and variance at test points.
//
// The mean is the rectangular kernel product K_hat(test, train) w.  The
// variance var_j = k(x*_j, x*_j) - k_j^T (K_hat + gamma I)^{-1} k_j needs one
// solve per test point with right-hand side k_j = K_hat(train, x*_j): the test
// points go 16 at a time, their columns k_j formed explicitly (an n x 16 block),
// solved together as one multi-right-hand-side system, and each column's
// quadratic form reduced in a fixed order.  k(x, x) = 1 for both kernels.
#include "krr_internal.h"

namespace krr {

namespace {

constexpr int PBATCH = 16;

__device__ __forceinline__ double kval(const double *a, const double *b, int d, double sigma, int kernel) {
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double t = a[k] - b[k];
        r2 = fma(t, t, r2);
    }
    if (kernel == KRR_KERNEL_MATERN32) {
        const double s = sqrt(3.0 * r2) / sigma;
        return (1.0 + s) * exp(-s);
    }
    return exp(-r2 / (2.0 * sigma * sigma));
}

// B[i + c n] = k(x_i, xs_{j0 + c}) for the batch's columns, 0 beyond the last test point.
__global__ __launch_bounds__(BLOCK) void k_kernel_block(const double *__restrict__ x, int64_t n, int d,
                                                        const double *__restrict__ xs, int64_t m, int64_t j0,
                                                        double sigma, int kernel, double *B) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(BLOCK) + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    const int64_t j = j0 + c;
    B[i + c * n] = (j < m) ? kval(x + i * d, xs + j * d, d, sigma, kernel) : 0.0;
}

// var[j0 + c] = 1 - sum_i B[i + c n] W[i + c n] (one block per column).
__global__ __launch_bounds__(BLOCK) void k_var_block(const double *__restrict__ B, const double *__restrict__ W,
                                                     int64_t n, int64_t m, int64_t j0, double *var) {
    __shared__ double sh[BLOCK];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += BLOCK) s = fma(B[i + c * n], W[i + c * n], s);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w /= 2) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && j0 + c < m) var[j0 + c] = 1.0 - sh[0];
}

}  // namespace

size_t predict_var_bytes(int64_t n) { return align_up(static_cast<size_t>(n) * PBATCH * 8, 256) * 2; }

hipError_t predict_kernel_block(const double *x, int64_t n, int d, const double *xs, int64_t m, int64_t j0,
                                double sigma, int kernel, double *B, hipStream_t s) {
    hipLaunchKernelGGL(k_kernel_block, dim3((n + BLOCK - 1) / BLOCK, PBATCH), dim3(BLOCK), 0, s, x, n, d, xs, m, j0,
                       sigma, kernel, B);
    return hipGetLastError();
}

hipError_t predict_var_block(const double *B, const double *W, int64_t n, int64_t m, int64_t j0, double *var,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_var_block, dim3(PBATCH), dim3(BLOCK), 0, s, B, W, n, m, j0, var);
    return hipGetLastError();
}

}  // namespace krr
