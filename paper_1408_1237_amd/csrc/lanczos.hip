// Extreme eigenvalues of a conjugate gradient run's Lanczos tridiagonal (host
// code only).  CG on a symmetric positive definite matrix builds the same
// Krylov basis as the Lanczos process; its step lengths alpha_j and residual
// ratios beta_j give the tridiagonal T_k whose extreme eigenvalues (Ritz
// values) estimate those of the matrix, and so the condition number that
// governs CG's convergence (section 3).
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/krr.h"

namespace {

// Number of eigenvalues of the symmetric tridiagonal (diag a, sub-diagonal e,
// e[0] unused) that are < x: negative pivots of the LDL^T factorisation of T - xI.
int sturm_below(const std::vector<double> &a, const std::vector<double> &e, double x) {
    int count = 0;
    double q = 1.0;
    const double tiny = 1e-300;
    for (size_t j = 0; j < a.size(); ++j) {
        q = (a[j] - x) - (j > 0 ? e[j] * e[j] / q : 0.0);
        if (q == 0.0) q = -tiny;
        if (q < 0.0) ++count;
    }
    return count;
}

// The idx-th smallest eigenvalue (0-based) in [lo, hi] by bisection.
double bisect(const std::vector<double> &a, const std::vector<double> &e, int idx, double lo, double hi) {
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, e, mid) > idx) hi = mid;
        else lo = mid;
        if (hi - lo <= 1e-15 * std::max(std::fabs(lo), std::fabs(hi))) break;
    }
    return 0.5 * (lo + hi);
}

}  // namespace

extern "C" int krr_lanczos_extremes(const double *alpha, const double *beta, int32_t k, double *lambda_min,
                                    double *lambda_max) {
    if (alpha == nullptr || beta == nullptr || lambda_min == nullptr || lambda_max == nullptr || k < 1)
        return KRR_EINVAL;
    for (int j = 0; j < k; ++j) {
        if (!std::isfinite(alpha[j]) || !(alpha[j] > 0.0)) return KRR_EINVAL;
        if (j + 1 < k && (!std::isfinite(beta[j]) || beta[j] < 0.0)) return KRR_EINVAL;
    }
    std::vector<double> a(k), e(k, 0.0);
    a[0] = 1.0 / alpha[0];
    for (int j = 1; j < k; ++j) {
        a[j] = 1.0 / alpha[j] + beta[j - 1] / alpha[j - 1];
        e[j] = std::sqrt(beta[j - 1]) / alpha[j - 1];
    }
    // Gershgorin interval of T
    double lo = a[0], hi = a[0];
    for (int j = 0; j < k; ++j) {
        const double r = e[j] + (j + 1 < k ? e[j + 1] : 0.0);
        lo = std::min(lo, a[j] - r);
        hi = std::max(hi, a[j] + r);
    }
    const double pad = 1e-12 * std::max(std::fabs(lo), std::fabs(hi)) + 1e-300;
    lo -= pad;
    hi += pad;
    *lambda_min = bisect(a, e, 0, lo, hi);
    *lambda_max = bisect(a, e, k - 1, lo, hi);
    return KRR_OK;
}
