// C ABI entry points (include/krr.h): argument validation, workspace layout,
// point preparation and dispatch to the kernels and solver drivers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "solvers.h"

using namespace krr;

namespace {

constexpr int64_t kMaxN = (int64_t(1) << 31) - 2 * TILE;

bool is_fin(double v) { return std::isfinite(v); }

int check_points(const krr_points *p) {
    if (p == nullptr || p->x == nullptr) return KRR_EINVAL;
    if (p->n < 1 || p->n > kMaxN) return KRR_EINVAL;
    if (p->d < 1 || p->d > KRR_MAX_DIM) return KRR_EINVAL;
    return KRR_OK;
}

int check_sigma(double sigma) { return (is_fin(sigma) && sigma > 0.0) ? KRR_OK : KRR_EINVAL; }

int check_prec(int32_t prec) { return (prec == KRR_FP64 || prec == KRR_FP32 || prec == KRR_BF16) ? KRR_OK : KRR_EINVAL; }

// Resolve the options: defaults of section 6 for negative fields.
int resolve_opts(const krr_fgmres_opts *in, double gamma, SolverOpts &o) {
    krr_fgmres_opts d;
    krr_default_opts(&d);
    const krr_fgmres_opts &u = in ? *in : d;
    o.restart_m = u.restart_m < 0 ? d.restart_m : u.restart_m;
    o.max_outer = u.max_outer < 0 ? d.max_outer : u.max_outer;
    o.tol = u.tol < 0 ? d.tol : u.tol;
    o.inner = u.inner;
    o.inner_prec = u.inner_prec < 0 ? d.inner_prec : u.inner_prec;
    o.delta = u.delta < 0 ? (gamma > 0.0 ? 10.0 * gamma : 1e-3) : u.delta;
    o.inner_maxit = u.inner_maxit < 0 ? d.inner_maxit : u.inner_maxit;
    o.inner_tol = u.inner_tol < 0 ? 10.0 * o.tol : u.inner_tol;
    o.gs = u.gs < 0 ? d.gs : u.gs;
    o.cg_check = u.cg_check <= 0 ? d.cg_check : u.cg_check;
    o.kernel = u.kernel;
    if (o.restart_m < 1 || o.restart_m > 1000) return KRR_EINVAL;
    if (o.max_outer < 1) return KRR_EINVAL;
    if (!is_fin(o.tol) || o.tol <= 0.0) return KRR_EINVAL;
    if (o.inner != KRR_INNER_CG && o.inner != KRR_INNER_NONE) return KRR_EINVAL;
    if (check_prec(o.inner_prec) != KRR_OK) return KRR_EINVAL;
    if (!is_fin(o.delta) || o.delta < 0.0) return KRR_EINVAL;
    if (o.inner == KRR_INNER_CG && o.inner_maxit < 1) return KRR_EINVAL;
    if (!is_fin(o.inner_tol) || o.inner_tol < 0.0) return KRR_EINVAL;
    if (o.gs != KRR_GS_MGS && o.gs != KRR_GS_CGS2) return KRR_EINVAL;
    if (o.kernel != KRR_KERNEL_GAUSS && o.kernel != KRR_KERNEL_MATERN32) return KRR_EINVAL;
    return KRR_OK;
}

// Everything one single-system call carves from the workspace, in order.
struct Layout {
    Prepared P;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    SolverWork W;
    void *q = nullptr, *y = nullptr;   // kmvp: sorted q and y (8 bytes per entry)
    uint16_t *q16 = nullptr;
    size_t total = 0;
};

enum Kind { K_MVP, K_INNER, K_FGMRES, K_CG64 };

Layout carve(void *ws, int64_t n, int d, const SolverOpts &o, Kind kind) {
    Carver cv(ws);
    Layout L;
    L.P = carve_prepared(cv, n, d);
    L.temp_bytes = prep_temp_bytes(n);
    L.temp = cv.take<char>(L.temp_bytes);
    if (kind == K_MVP) {
        L.q = cv.take<double>(L.P.n_pad);
        L.y = cv.take<double>(L.P.n_pad);
        L.q16 = cv.take<uint16_t>(L.P.n_pad);
        L.W.ksc = carve_kmvp_scratch(cv, L.P);
    } else {
        L.W = carve_solver(cv, L.P, o, kind == K_FGMRES || kind == K_INNER);
    }
    L.total = cv.off + 256;
    return L;
}

size_t layout_bytes(int64_t n, int d, const SolverOpts &o, Kind kind) { return carve(nullptr, n, d, o, kind).total; }

// Several right-hand sides: one prepared set and the product scratch.
struct MultiLayout {
    Prepared P;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    void *scratch = nullptr;
    size_t total = 0;
};

MultiLayout carve_multi(void *ws, int64_t n, int d, int nrhs) {
    Carver cv(ws);
    MultiLayout L;
    L.P = carve_prepared(cv, n, d);
    L.temp_bytes = prep_temp_bytes(n);
    L.temp = cv.take<char>(L.temp_bytes);
    L.scratch = cv.take<char>(kmvp_multi_scratch_bytes(L.P, nrhs));
    L.total = cv.off + 256;
    return L;
}

// Gradient pass: one prepared set and the pass's scratch.
struct GradLayout {
    Prepared P;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    void *scratch = nullptr;
    size_t total = 0;
};

GradLayout carve_grad(void *ws, int64_t n, int d) {
    Carver cv(ws);
    GradLayout L;
    L.P = carve_prepared(cv, n, d);
    L.temp_bytes = prep_temp_bytes(n);
    L.temp = cv.take<char>(L.temp_bytes);
    L.scratch = cv.take<char>(grad_scratch_bytes(L.P));
    L.total = cv.off + 256;
    return L;
}

// Rectangular product: two prepared sets, one preparation scratch (reused).
struct CrossLayout {
    Prepared T, S;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    void *q = nullptr, *y = nullptr;
    uint16_t *q16 = nullptr;
    KmvpScratch ksc;
    size_t total = 0;
};

CrossLayout carve_cross(void *ws, int64_t nt, int64_t ns, int d) {
    Carver cv(ws);
    CrossLayout L;
    L.T = carve_prepared(cv, nt, d);
    L.S = carve_prepared(cv, ns, d);
    L.temp_bytes = prep_temp_bytes(nt > ns ? nt : ns);
    L.temp = cv.take<char>(L.temp_bytes);
    L.q = cv.take<double>(L.S.n_pad);
    L.y = cv.take<double>(L.T.n_pad);
    L.q16 = cv.take<uint16_t>(L.S.n_pad);
    L.ksc = carve_kmvp_cross_scratch(cv, L.T, L.S);
    L.total = cv.off + 256;
    return L;
}

// Align the caller's workspace to 256 bytes.
void *align_ws(void *ws, size_t &bytes) {
    const uintptr_t p = reinterpret_cast<uintptr_t>(ws);
    const uintptr_t a = (p + 255) / 256 * 256;
    if (a - p > bytes) {
        bytes = 0;
        return ws;
    }
    bytes -= (a - p);
    return reinterpret_cast<void *>(a);
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

void krr_default_opts(krr_fgmres_opts *o) {
    if (!o) return;
    o->restart_m = 30;
    o->max_outer = 1000;
    o->tol = 1e-6;
    o->inner = KRR_INNER_CG;
    o->inner_prec = KRR_FP32;
    o->delta = -1.0;
    o->inner_maxit = 10;
    o->inner_tol = -1.0;
    o->gs = KRR_GS_MGS;
    o->cg_check = 16;
    o->kernel = KRR_KERNEL_GAUSS;
}

const char *krr_status_string(int s) {
    switch (s) {
        case KRR_OK: return "KRR_OK";
        case KRR_NOT_CONVERGED: return "KRR_NOT_CONVERGED";
        case KRR_BREAKDOWN: return "KRR_BREAKDOWN";
        case KRR_EINVAL: return "KRR_EINVAL: invalid argument";
        case KRR_ENONFINITE: return "KRR_ENONFINITE: non-finite input";
        case KRR_EWORKSPACE: return "KRR_EWORKSPACE: workspace missing or too small";
        case KRR_EHIP: return "KRR_EHIP: HIP runtime error";
        case KRR_EUNSUPPORTED: return "KRR_EUNSUPPORTED";
        default: return "unknown status";
    }
}

size_t krr_workspace_size(int32_t which, const krr_points *probs, int32_t nprob, int32_t nrhs,
                          const krr_fgmres_opts *opts) {
    if (probs == nullptr || nprob < 1) return 0;
    SolverOpts o;
    if (resolve_opts(opts, 0.0, o) != KRR_OK) return 0;
    switch (which) {
        case KRR_WS_KMVP:
            if (probs[0].n < 1 || probs[0].d < 1 || probs[0].d > KRR_MAX_DIM) return 0;
            return layout_bytes(probs[0].n, probs[0].d, o, K_MVP) + 256;
        case KRR_WS_KMVP_GRAD:
            if (probs[0].n < 1 || probs[0].d < 1 || probs[0].d > KRR_MAX_DIM) return 0;
            return carve_grad(nullptr, probs[0].n, probs[0].d).total + 256;
        case KRR_WS_KMVP_MULTI:
            if (probs[0].n < 1 || probs[0].d < 1 || probs[0].d > KRR_MAX_DIM || nrhs < 1 || nrhs > 4096) return 0;
            return carve_multi(nullptr, probs[0].n, probs[0].d, nrhs).total + 256;
        case KRR_WS_CG_INNER:
            if (probs[0].n < 1 || probs[0].d < 1 || probs[0].d > KRR_MAX_DIM) return 0;
            return layout_bytes(probs[0].n, probs[0].d, o, K_INNER) + 256;
        case KRR_WS_FGMRES:
            if (probs[0].n < 1 || probs[0].d < 1 || probs[0].d > KRR_MAX_DIM) return 0;
            return layout_bytes(probs[0].n, probs[0].d, o, K_FGMRES) + 256;
        case KRR_WS_KMVP_CROSS:
            if (nprob < 2) return 0;
            for (int k = 0; k < 2; ++k)
                if (probs[k].n < 1 || probs[k].d < 1 || probs[k].d > KRR_MAX_DIM) return 0;
            if (probs[0].d != probs[1].d) return 0;
            return carve_cross(nullptr, probs[0].n, probs[1].n, probs[0].d).total + 256;
        case KRR_WS_PREDICT: {
            if (nprob < 2) return 0;
            for (int k = 0; k < 2; ++k)
                if (probs[k].n < 1 || probs[k].d < 1 || probs[k].d > KRR_MAX_DIM) return 0;
            if (probs[0].d != probs[1].d) return 0;
            const size_t cross = carve_cross(nullptr, probs[1].n, probs[0].n, probs[0].d).total;
            const size_t solve = krr_workspace_size(KRR_WS_SOLVE, probs, 1, 16, opts);
            if (solve == 0) return 0;
            const size_t var = predict_var_bytes(probs[0].n) + solve;
            return (cross > var ? cross : var) + 512;
        }
        case KRR_WS_SOLVE: {
            if (nrhs < 1) return 0;
            size_t mx = 0;
            for (int k = 0; k < nprob; ++k) {
                if (probs[k].n < 1 || probs[k].d < 1 || probs[k].d > KRR_MAX_DIM) return 0;
                // every mode's single solve: the flexible solvers' basis, or the
                // plain CG's coefficient history (2 max_outer values)
                const size_t b = std::max(layout_bytes(probs[k].n, probs[k].d, o, K_FGMRES),
                                          layout_bytes(probs[k].n, probs[k].d, o, K_CG64));
                if (b > mx) mx = b;
            }
            if (nprob > 1 || nrhs > 1) {
                const size_t bb = batch_workspace_bytes(probs, nprob, nrhs, o.restart_m);
                if (bb > mx) mx = bb;
            }
            return mx + 256;
        }
        default: return 0;
    }
}

// tune: time the launch shapes on the first product of a shape (kmvp_tune);
// false keeps the cached or default shape (no events, no synchronisation).
static int kmvp_single(const krr_points *pts, int kernel, double sigma, double shift, int32_t prec, const void *q,
                       void *y, void *ws, size_t ws_bytes, krr_stream_t stream, bool tune = true) {
    int rc;
    if ((rc = check_points(pts)) || (rc = check_sigma(sigma)) || (rc = check_prec(prec))) return rc;
    if (!is_fin(shift) || q == nullptr || y == nullptr || q == y) return KRR_EINVAL;
    if (ws == nullptr) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    SolverOpts o;
    Layout L = carve(nullptr, pts->n, pts->d, o, K_MVP);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve(ws, pts->n, pts->d, o, K_MVP);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KRR_HIP_STATUS(prepare_points(L.P, pts->x, sigma, L.temp, L.temp_bytes, s, kernel));
    if (prec == KRR_FP64) {
        KRR_HIP_STATUS((gather_sorted<double, double>(L.P, static_cast<const double *>(q), static_cast<double *>(L.q), s)));
        if (tune) KRR_HIP_STATUS(kmvp_tune(L.P, prec, L.q, L.y, L.W.ksc, s));
        KRR_HIP_STATUS(kmvp_sorted(L.P, prec, shift, L.q, L.y, L.W.ksc, nullptr, s));
        KRR_HIP_STATUS((scatter_sorted<double, double>(L.P, static_cast<double *>(L.y), static_cast<double *>(y), s)));
    } else {
        float *qs = static_cast<float *>(L.q);
        KRR_HIP_STATUS((gather_sorted<float, float>(L.P, static_cast<const float *>(q), qs, s)));
        const void *qin = qs;
        if (prec == KRR_BF16) {
            KRR_HIP_STATUS(to_bf16(qs, L.q16, L.P.n_pad, s));
            qin = L.q16;
        }
        if (tune) KRR_HIP_STATUS(kmvp_tune(L.P, prec, qin, L.y, L.W.ksc, s));
        KRR_HIP_STATUS(kmvp_sorted(L.P, prec, shift, qin, L.y, L.W.ksc, nullptr, s));
        KRR_HIP_STATUS((scatter_sorted<float, float>(L.P, static_cast<float *>(L.y), static_cast<float *>(y), s)));
    }
    return KRR_OK;
}

int kmvp_gauss(const krr_points *pts, double sigma, double shift, int32_t prec, const void *q, void *y, void *ws,
               size_t ws_bytes, krr_stream_t stream) {
    return kmvp_single(pts, KRR_KERNEL_GAUSS, sigma, shift, prec, q, y, ws, ws_bytes, stream);
}

int kmvp_matern(const krr_points *pts, double h, double shift, int32_t prec, const void *q, void *y, void *ws,
                size_t ws_bytes, krr_stream_t stream) {
    return kmvp_single(pts, KRR_KERNEL_MATERN32, h, shift, prec, q, y, ws, ws_bytes, stream);
}

}  // extern "C"

// The allocation-free product's body (noalloc.hip): kmvp_gauss on a given
// scratch, without tuning.
int kmvp_gauss_on_scratch(const krr_points *pts, double sigma, double shift, int32_t prec, const void *q, void *y,
                          void *scratch, size_t scratch_bytes, krr_stream_t stream) {
    return kmvp_single(pts, KRR_KERNEL_GAUSS, sigma, shift, prec, q, y, scratch, scratch_bytes, stream, false);
}

extern "C" {

int kmvp_gauss_multi(const krr_points *pts, double sigma, double shift, int32_t prec, int32_t nrhs, const void *Q,
                     int64_t ldq, void *Y, int64_t ldy, void *ws, size_t ws_bytes, krr_stream_t stream) {
    int rc;
    if ((rc = check_points(pts)) || (rc = check_sigma(sigma)) || (rc = check_prec(prec))) return rc;
    if (!is_fin(shift) || Q == nullptr || Y == nullptr || Q == Y || nrhs < 1 || nrhs > 4096 || ldq < pts->n ||
        ldy < pts->n)
        return KRR_EINVAL;
    if (ws == nullptr) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    MultiLayout L = carve_multi(nullptr, pts->n, pts->d, nrhs);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve_multi(ws, pts->n, pts->d, nrhs);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KRR_HIP_STATUS(prepare_points(L.P, pts->x, sigma, L.temp, L.temp_bytes, s));
    KRR_HIP_STATUS(kmvp_multi(L.P, prec, nrhs, shift, L.P.perm, Q, ldq, Y, ldy, L.scratch, s));
    return KRR_OK;
}

static int kmvp_cross_impl(const krr_points *targets, const krr_points *sources, int kernel, double sigma,
                           int32_t prec, const void *q, void *y, void *ws, size_t ws_bytes, krr_stream_t stream) {
    int rc;
    if ((rc = check_points(targets)) || (rc = check_points(sources)) || (rc = check_sigma(sigma)) ||
        (rc = check_prec(prec)))
        return rc;
    if (targets->d != sources->d || q == nullptr || y == nullptr || q == y) return KRR_EINVAL;
    if (ws == nullptr) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    CrossLayout L = carve_cross(nullptr, targets->n, sources->n, targets->d);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve_cross(ws, targets->n, sources->n, targets->d);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KRR_HIP_STATUS(prepare_points(L.T, targets->x, sigma, L.temp, L.temp_bytes, s, kernel));
    KRR_HIP_STATUS(prepare_points(L.S, sources->x, sigma, L.temp, L.temp_bytes, s, kernel));
    if (prec == KRR_FP64) {
        KRR_HIP_STATUS((gather_sorted<double, double>(L.S, static_cast<const double *>(q), static_cast<double *>(L.q), s)));
        KRR_HIP_STATUS(kmvp_cross_sorted(L.T, L.S, prec, L.q, L.y, L.ksc, s));
        KRR_HIP_STATUS((scatter_sorted<double, double>(L.T, static_cast<double *>(L.y), static_cast<double *>(y), s)));
    } else {
        float *qs = static_cast<float *>(L.q);
        KRR_HIP_STATUS((gather_sorted<float, float>(L.S, static_cast<const float *>(q), qs, s)));
        const void *qin = qs;
        if (prec == KRR_BF16) {
            KRR_HIP_STATUS(to_bf16(qs, L.q16, L.S.n_pad, s));
            qin = L.q16;
        }
        KRR_HIP_STATUS(kmvp_cross_sorted(L.T, L.S, prec, qin, L.y, L.ksc, s));
        KRR_HIP_STATUS((scatter_sorted<float, float>(L.T, static_cast<float *>(L.y), static_cast<float *>(y), s)));
    }
    return KRR_OK;
}

int kmvp_gauss_cross(const krr_points *targets, const krr_points *sources, double sigma, int32_t prec,
                     const void *q, void *y, void *ws, size_t ws_bytes, krr_stream_t stream) {
    return kmvp_cross_impl(targets, sources, KRR_KERNEL_GAUSS, sigma, prec, q, y, ws, ws_bytes, stream);
}

int kmvp_grad(const krr_points *pts, double sigma, double gamma, int32_t prec, const double *lam, const double *w,
              double *gx, double *g_logsigma, double *g_loggamma, void *ws, size_t ws_bytes, krr_stream_t stream) {
    int rc;
    if ((rc = check_points(pts)) || (rc = check_sigma(sigma))) return rc;
    if (prec != KRR_FP64 && prec != KRR_FP32) return KRR_EINVAL;
    if (!is_fin(gamma) || gamma < 0.0 || lam == nullptr || w == nullptr || gx == nullptr || g_logsigma == nullptr ||
        g_loggamma == nullptr)
        return KRR_EINVAL;
    if (ws == nullptr) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    GradLayout L = carve_grad(nullptr, pts->n, pts->d);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve_grad(ws, pts->n, pts->d);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KRR_HIP_STATUS(prepare_points(L.P, pts->x, sigma, L.temp, L.temp_bytes, s));
    KRR_HIP_STATUS(kmvp_grad_run(L.P, prec, sigma, gamma, lam, w, gx, g_logsigma, g_loggamma, L.scratch, s));
    return KRR_OK;
}

int cg_inner_solve(const krr_points *pts, double sigma, double shift, int32_t prec, const void *v, void *z,
                   int32_t maxit, double tol, krr_info *info, void *ws, size_t ws_bytes, krr_stream_t stream) {
    int rc;
    if ((rc = check_points(pts)) || (rc = check_sigma(sigma)) || (rc = check_prec(prec))) return rc;
    if (!is_fin(shift) || shift < 0.0 || v == nullptr || z == nullptr || maxit < 1 || !is_fin(tol) || tol < 0.0)
        return KRR_EINVAL;
    if (ws == nullptr) return KRR_EWORKSPACE;
    const double t0 = now_ms();
    ws = align_ws(ws, ws_bytes);
    SolverOpts o;
    Layout L = carve(nullptr, pts->n, pts->d, o, K_INNER);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve(ws, pts->n, pts->d, o, K_INNER);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KRR_HIP_STATUS(prepare_points(L.P, pts->x, sigma, L.temp, L.temp_bytes, s));
    if (prec == KRR_FP64)
        KRR_HIP_STATUS((gather_sorted<double, double>(L.P, static_cast<const double *>(v), L.W.b, s)));
    else
        KRR_HIP_STATUS((gather_sorted<float, double>(L.P, static_cast<const float *>(v), L.W.b, s)));
    if (info) std::memset(info, 0, sizeof(*info));
    rc = cg_inner_sorted(L.P, prec, shift, L.W.b, L.W.x, maxit, tol, L.W, info, s);
    if (rc < 0) return rc;
    if (prec == KRR_FP64)
        KRR_HIP_STATUS((scatter_sorted<double, double>(L.P, L.W.x, static_cast<double *>(z), s)));
    else
        KRR_HIP_STATUS((scatter_sorted<double, float>(L.P, L.W.x, static_cast<float *>(z), s)));
    if (info) {
        KRR_HIP_STATUS(hipStreamSynchronize(s));
        info->t_total_ms = now_ms() - t0;
    }
    return rc;
}

static int solve_one(const krr_points *pts, double sigma, double gamma, const double *b, double *x, bool x0_zero,
                     int mode, const SolverOpts &o, krr_info *info, void *ws, size_t ws_bytes, hipStream_t s) {
    const double t0 = now_ms();
    const Kind kind = (mode == KRR_MODE_CG64) ? K_CG64 : K_FGMRES;
    Layout L = carve(nullptr, pts->n, pts->d, o, kind);
    if (L.total > ws_bytes) return KRR_EWORKSPACE;
    L = carve(ws, pts->n, pts->d, o, kind);
    KRR_HIP_STATUS(prepare_points(L.P, pts->x, sigma, L.temp, L.temp_bytes, s, o.kernel));
    int flags = 0;
    KRR_HIP_STATUS(hipMemcpyAsync(&flags, L.P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    KRR_HIP_STATUS(hipStreamSynchronize(s));
    if (flags & 1) return KRR_ENONFINITE;
    const double t_prep = now_ms() - t0;
    KRR_HIP_STATUS((gather_sorted<double, double>(L.P, b, L.W.b, s)));
    if (!x0_zero) KRR_HIP_STATUS((gather_sorted<double, double>(L.P, x, L.W.x, s)));
    else KRR_HIP_STATUS(fill_d(L.W.x, L.P.n_pad, 0.0, s));
    krr_info tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    int rc;
    if (mode == KRR_MODE_CG64) {
        rc = cg64_sorted(L.P, gamma, o, L.W, &tmp, s);
    } else if (mode == KRR_MODE_FCG) {
        rc = fcg_sorted(L.P, gamma, o, L.W, &tmp, s);
    } else {
        SolverOpts oo = o;
        if (mode == KRR_MODE_GMRES) oo.inner = KRR_INNER_NONE;
        rc = fgmres_sorted(L.P, gamma, x0_zero, oo, L.W, &tmp, s);
    }
    if (rc < 0) return rc;
    KRR_HIP_STATUS((scatter_sorted<double, double>(L.P, L.W.x, x, s)));
    KRR_HIP_STATUS(hipStreamSynchronize(s));
    tmp.t_total_ms = now_ms() - t0;
    tmp.t_prep_ms = t_prep;
    tmp.status = rc;
    if (info) *info = tmp;
    return rc;
}

int fgmres_solve(const krr_points *pts, double sigma, double gamma, const double *b, double *x,
                 const krr_fgmres_opts *opts, krr_info *info, void *ws, size_t ws_bytes, krr_stream_t stream) {
    int rc;
    if ((rc = check_points(pts)) || (rc = check_sigma(sigma))) return rc;
    if (!is_fin(gamma) || gamma < 0.0 || b == nullptr || x == nullptr || b == x) return KRR_EINVAL;
    SolverOpts o;
    if ((rc = resolve_opts(opts, gamma, o)) != KRR_OK) return rc;
    if (ws == nullptr) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    return solve_one(pts, sigma, gamma, b, x, false, KRR_MODE_FGMRES, o, info, ws, ws_bytes,
                     reinterpret_cast<hipStream_t>(stream));
}

int krr_solve(const krr_points *probs, int32_t nprob, const double *sigma, const double *gamma, int32_t nrhs,
              const double *const *Y, const int64_t *ldy, double *const *W, int32_t mode,
              const krr_fgmres_opts *opts, krr_info *infos, void *ws, size_t ws_bytes, krr_stream_t stream) {
    if (probs == nullptr || nprob < 1 || sigma == nullptr || gamma == nullptr || nrhs < 1 || Y == nullptr ||
        W == nullptr)
        return KRR_EINVAL;
    if (mode != KRR_MODE_FGMRES && mode != KRR_MODE_CG64 && mode != KRR_MODE_GMRES && mode != KRR_MODE_FCG)
        return KRR_EINVAL;
    int rc;
    for (int k = 0; k < nprob; ++k) {
        if ((rc = check_points(&probs[k])) || (rc = check_sigma(sigma[k]))) return rc;
        if (!is_fin(gamma[k]) || gamma[k] < 0.0 || Y[k] == nullptr || W[k] == nullptr) return KRR_EINVAL;
        if (ldy && ldy[k] < probs[k].n) return KRR_EINVAL;
        SolverOpts o;
        if ((rc = resolve_opts(opts, gamma[k], o)) != KRR_OK) return rc;
    }
    if (ws == nullptr) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    SolverOpts o0;
    resolve_opts(opts, gamma[0], o0);
    const bool several = nprob > 1 || nrhs > 1;
    const bool fp64_inner = mode == KRR_MODE_FGMRES && o0.inner == KRR_INNER_CG && o0.inner_prec == KRR_FP64;
    if ((mode == KRR_MODE_FGMRES || mode == KRR_MODE_GMRES) && several && o0.kernel == KRR_KERNEL_GAUSS &&
        !fp64_inner) {
        // all systems and columns advance together (one product launch per
        // dimension class per step for all columns, per-column solver state on
        // the device)
        SolverOpts o;
        resolve_opts(opts, gamma[0], o);
        o.delta = (opts && opts->delta >= 0) ? opts->delta : -1.0;  // per system: 10 gamma_k
        if (mode == KRR_MODE_GMRES) o.inner = KRR_INNER_NONE;
        return batched_fgmres(probs, nprob, sigma, gamma, nrhs, Y, ldy, W, o, infos, ws, ws_bytes, s);
    }
    if (mode == KRR_MODE_CG64 && several && o0.kernel == KRR_KERNEL_GAUSS) {
        SolverOpts o;
        resolve_opts(opts, gamma[0], o);
        return batched_cg64(probs, nprob, sigma, gamma, nrhs, Y, ldy, W, o, infos, ws, ws_bytes, s);
    }
    int worst = KRR_OK;
    for (int k = 0; k < nprob; ++k) {
        SolverOpts o;
        resolve_opts(opts, gamma[k], o);
        const int64_t ld = ldy ? ldy[k] : probs[k].n;
        for (int r = 0; r < nrhs; ++r) {
            krr_info *inf = infos ? &infos[static_cast<size_t>(k) * nrhs + r] : nullptr;
            rc = solve_one(&probs[k], sigma[k], gamma[k], Y[k] + static_cast<size_t>(r) * ld,
                           W[k] + static_cast<size_t>(r) * ld, true, mode, o, inf, ws, ws_bytes, s);
            if (rc < 0) return rc;
            if (rc > worst) worst = rc;
        }
    }
    return worst;
}

int krr_predict(const krr_points *train, const krr_points *test, double sigma, double gamma, const double *w,
                double *mean, double *var, const krr_fgmres_opts *opts, krr_info *infos, void *ws, size_t ws_bytes,
                krr_stream_t stream) {
    int rc;
    if ((rc = check_points(train)) || (rc = check_points(test)) || (rc = check_sigma(sigma))) return rc;
    if (train->d != test->d || !is_fin(gamma) || gamma < 0.0 || w == nullptr || mean == nullptr) return KRR_EINVAL;
    SolverOpts o;
    if ((rc = resolve_opts(opts, gamma, o)) != KRR_OK) return rc;
    const krr_points probs[2] = {*train, *test};
    const size_t need = krr_workspace_size(KRR_WS_PREDICT, probs, 2, 1, opts);
    if (ws == nullptr || need == 0 || ws_bytes < need) return KRR_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // mean = K_hat(test, train) w (FP64)
    if ((rc = kmvp_cross_impl(test, train, o.kernel, sigma, KRR_FP64, w, mean, ws, ws_bytes, stream)) != KRR_OK)
        return rc;
    if (var == nullptr) return KRR_OK;
    // variance: 16 test points per multi-right-hand-side solve
    void *base = align_ws(ws, ws_bytes);
    const int64_t n = train->n, m = test->n;
    Carver cv(base);
    double *B = cv.take<double>(static_cast<size_t>(n) * 16);
    double *Wb = cv.take<double>(static_cast<size_t>(n) * 16);
    void *sws = cv.take<char>(0);
    const size_t sbytes = ws_bytes - cv.off;
    krr_fgmres_opts oo;
    if (opts) oo = *opts;
    else krr_default_opts(&oo);
    int worst = KRR_OK;
    krr_info binfo[16];
    for (int64_t j0 = 0; j0 < m; j0 += 16) {
        KRR_HIP_STATUS(predict_kernel_block(train->x, n, train->d, test->x, m, j0, sigma, o.kernel, B, s));
        const double *Yp[1] = {B};
        double *Wp[1] = {Wb};
        const int64_t ld[1] = {n};
        rc = krr_solve(train, 1, &sigma, &gamma, 16, Yp, ld, Wp, KRR_MODE_FGMRES, &oo, binfo, sws, sbytes, stream);
        if (rc < 0) return rc;
        KRR_HIP_STATUS(predict_var_block(B, Wb, n, m, j0, var, s));
        for (int c = 0; c < 16 && j0 + c < m; ++c) {
            if (infos) infos[j0 + c] = binfo[c];
            if (binfo[c].status > worst) worst = binfo[c].status;
        }
    }
    return worst;
}

int krr_profile_begin(int32_t max_launches) { return profile_begin(max_launches); }

int krr_profile_end(krr_profile_stats *out) { return profile_end(out); }

size_t krr_probe_workspace_size(void) { return probe_workspace_bytes() + 256; }

int krr_probe_issue_rates(double *rates, void *ws, size_t ws_bytes, krr_stream_t stream) {
    if (rates == nullptr) return KRR_EINVAL;
    if (ws == nullptr || ws_bytes < krr_probe_workspace_size()) return KRR_EWORKSPACE;
    ws = align_ws(ws, ws_bytes);
    KRR_HIP_STATUS(probe_issue_rates(rates, ws, reinterpret_cast<hipStream_t>(stream)));
    return KRR_OK;
}

}  // extern "C"
