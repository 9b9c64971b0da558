/*
 * krr.h -- C ABI of the MI355X (gfx950) solver for regularised Gaussian kernel
 * systems (K_hat + gamma I) w = y, after Srinivasan, Hu, Gumerov, Murtugudde,
 * Duraiswami, "Preconditioned Krylov solvers for kernel regression".
 *
 * Problem statement (section 1, section 2): points X = {x_1..x_N} in R^d, the
 * Gaussian kernel k(x_i, x_j) = exp(-||x_i - x_j||^2 / (2 sigma^2))
 * (eq. Gaussian), the kernel matrix K_hat_ij = k(x_i, x_j) including the
 * diagonal (eq. kernelMatrix), and the regularised matrix K = K_hat + gamma I
 * (eq. RegKernel).  The solver is flexible GMRES (Algorithm 1, section 4.2),
 * right-preconditioned by M = K_hat + delta I (section 5) whose systems are
 * solved approximately by a truncated inner CG (sections 4.3, 5.2) with a
 * low-precision kernel product; the outer product is double precision
 * (section 5.1).  K_hat is never stored: every product is an on-the-fly
 * weighted kernel sum (section 1; section 3.1).
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers unless the comment says (host).  The caller
 *    owns every buffer, including the workspace `ws` of `ws_bytes` bytes; the
 *    library never allocates or frees device memory.  Required workspace sizes
 *    come from krr_workspace_size().
 *  - Points are n x d row-major FP64 (x[i*d + t]), read only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the default stream).
 *    The product and gradient calls are asynchronous.  The solvers read small
 *    status words back from the device (one per outer step, or per group of CG
 *    iterations) and therefore synchronise `stream`.
 *  - Return values: KRR_OK (0); positive values mean the call completed with
 *    a result but not the requested one (KRR_NOT_CONVERGED: the best iterate is
 *    in the output; KRR_BREAKDOWN: a non-positive curvature or non-finite value
 *    stopped a CG); negative values are errors.  Argument errors are detected on
 *    the host before anything is enqueued, and outputs are then untouched.
 *  - Non-finite inputs (NaN/Inf in points, right-hand sides or vectors) are
 *    reported as KRR_ENONFINITE by the solvers (detected on the device during
 *    set-up, before the iteration starts).
 *  - Calls that share a workspace must not overlap; different workspaces may
 *    be used concurrently on different streams.
 */
#ifndef KRR_H
#define KRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;
typedef struct ihipStream_t *krr_stream_t; /* same type as hipStream_t */

/* Arithmetic of a kernel product.  KRR_BF16 stores point offsets and the input
 * vector in bfloat16 (round to nearest even) and accumulates in FP32; its
 * vectors are FP32 in memory. */
typedef enum { KRR_FP64 = 0, KRR_FP32 = 1, KRR_BF16 = 2 } krr_prec;

typedef enum {
    KRR_OK = 0,
    KRR_NOT_CONVERGED = 1,
    KRR_BREAKDOWN = 2,
    KRR_EINVAL = -1,      /* bad argument (sizes, sigma <= 0, gamma < 0, NULL, ...) */
    KRR_ENONFINITE = -2,  /* NaN or Inf in an input */
    KRR_EWORKSPACE = -3,  /* ws NULL or ws_bytes below krr_workspace_size() */
    KRR_EHIP = -4,        /* a HIP runtime call failed */
    KRR_EUNSUPPORTED = -5 /* valid but not implemented (e.g. d above KRR_MAX_DIM) */
} krr_status;

#define KRR_MAX_DIM 64

/* One point set: n points of dimension d, n x d row-major FP64, device. */
typedef struct {
    int64_t n;
    int32_t d;
    const double *x;
} krr_points;

/* Inner preconditioner of the flexible solver. */
typedef enum {
    KRR_INNER_CG = 0,   /* truncated CG on M = K_hat + delta I (section 5) */
    KRR_INNER_NONE = 1  /* z_j = v_j: M = I, i.e. plain restarted GMRES */
} krr_inner;

/* Orthogonalisation of the Arnoldi vectors: modified Gram-Schmidt as printed
 * in Algorithm 1, or classical Gram-Schmidt applied twice. */
typedef enum { KRR_GS_MGS = 0, KRR_GS_CGS2 = 1 } krr_gs;

/* Kernel of K_hat: the Gaussian of eq. Gaussian (section 1), with sigma its
 * bandwidth, or the Matern kernel with smoothness 3/2 of eq. MaternKernel
 * (section 6), k = (1 + sqrt(3) d) exp(-sqrt(3) d), d = ||x_i - x_j|| / h, with
 * the length scale h passed where the calls take sigma.  The Matern kernel is
 * available in kmvp_matern and in the solvers (fgmres_solve, krr_solve; several
 * systems or columns are then solved one after the other); the multi-RHS, cross
 * and gradient calls are Gaussian. */
typedef enum { KRR_KERNEL_GAUSS = 0, KRR_KERNEL_MATERN32 = 1 } krr_kernel;

/* Options of the flexible solver.  krr_default_opts() fills the paper's rules
 * (section 6): outer tolerance 1e-6, inner tolerance ten times the outer
 * tolerance, delta ten times gamma (1e-3 when gamma = 0).  Fields with a
 * negative value take those defaults at call time. */
typedef struct {
    int32_t restart_m;   /* Krylov vectors per cycle ("iter" of Algorithm 1); default 30 */
    int32_t max_outer;   /* cap on outer steps over all cycles; default 1000 */
    double tol;          /* stop when ||y - K w|| / ||y|| <= tol (true FP64 residual) */
    int32_t inner;       /* krr_inner */
    int32_t inner_prec;  /* krr_prec of the inner products; default KRR_FP32 */
    double delta;        /* M = K_hat + delta I; < 0: 10 gamma, or 1e-3 if gamma == 0 */
    int32_t inner_maxit; /* inner CG iterations cap (>= 1); default 10 */
    double inner_tol;    /* inner stop at ||r|| / ||v|| <= inner_tol; < 0: 10 tol; 0: run to the cap */
    int32_t gs;          /* krr_gs; default KRR_GS_MGS */
    int32_t cg_check;    /* plain CG: iterations between host checks of the stop flag; several systems or
                            columns (krr_solve): also the outer steps between checks; default 16 */
    int32_t kernel;      /* krr_kernel of K_hat; default KRR_KERNEL_GAUSS */
} krr_fgmres_opts;

/* Per-solve report (host struct, caller-owned). */
typedef struct {
    int32_t status;        /* krr_status of this solve */
    int32_t outer_iters;   /* outer steps over all cycles (CG: iterations) */
    int32_t inner_iters;   /* inner CG iterations in total */
    int32_t cycles;        /* restart cycles (CG: true-residual restarts + 1) */
    int64_t mvp64, mvp32, mvp16; /* kernel products by precision */
    double relres_true;    /* ||y - K w|| / ||y|| from an FP64 product at exit */
    double relres_est;     /* the solver's own last estimate */
    double t_total_ms;     /* host wall time of the call */
    /* Plain CG (KRR_MODE_CG64) only, else 0: the smallest and largest eigenvalue
     * of K_hat + gamma I estimated from the first CG run's coefficients (the
     * extreme Ritz values of its Lanczos tridiagonal, krr_lanczos_extremes); their
     * ratio estimates the condition number that sets CG's convergence (section 3,
     * the need for preconditioning in section 5).  lambda_max_est converges in a
     * few iterations; lambda_min_est approaches the true value from above as CG
     * converges, so the ratio is a lower estimate of the condition number. */
    double lambda_min_est;
    double lambda_max_est;
    /* Where the time went (ms): point preparation (scaling, sort, tiles; for
     * several systems also the autotuning of the batched products), and for
     * fgmres_solve and single-column krr_solve calls in FGMRES mode the inner
     * solves, the outer FP64 products and the orthogonalisation with the Givens
     * update, from HIP events on the call's stream (0 where not measured). */
    double t_prep_ms;
    double t_inner_ms;
    double t_outer_ms;
    double t_ortho_ms;
    int32_t batch_steps;   /* several systems or columns: outer steps (CG: iterations) the batch ran, else 0 */
    int32_t batch_tiles;   /* several systems or columns: column tiles per work item of the batched
                              products (autotuned once per process; first dimension class), else 0 */
} krr_info;

/* Solver modes of krr_solve. */
typedef enum {
    KRR_MODE_FGMRES = 0, /* mixed precision flexible GMRES (the paper's method) */
    KRR_MODE_CG64 = 1,   /* plain FP64 conjugate gradient (the paper's baseline) */
    KRR_MODE_GMRES = 2,  /* FGMRES with inner = KRR_INNER_NONE */
    KRR_MODE_FCG = 3     /* flexible CG (sections 4.2, 5.4): each new direction K-orthogonalised
                            against up to restart_m - 1 previous ones, same inner solver */
} krr_mode;

/* Which call a workspace is sized for (krr_workspace_size). */
typedef enum {
    KRR_WS_KMVP = 0,
    KRR_WS_KMVP_MULTI = 1,
    KRR_WS_KMVP_GRAD = 2,
    KRR_WS_CG_INNER = 3,
    KRR_WS_FGMRES = 4,
    KRR_WS_SOLVE = 5,
    KRR_WS_KMVP_CROSS = 6,
    KRR_WS_PREDICT = 7
} krr_ws_call;

void krr_default_opts(krr_fgmres_opts *opts /* host */);
const char *krr_status_string(int status);

/* Bytes of workspace needed by call `which` for the given problem(s).
 * probs: host array of nprob point sets (only n and d are read); for
 * KRR_WS_KMVP_CROSS probs[0] are the targets and probs[1] the sources, for
 * KRR_WS_PREDICT probs[0] the training and probs[1] the test points.  nrhs is
 * the number of right-hand sides (multi products, krr_solve).  opts may be NULL
 * (defaults).  Returns 0 for invalid arguments. */
size_t krr_workspace_size(int32_t which, const krr_points *probs, int32_t nprob, int32_t nrhs,
                          const krr_fgmres_opts *opts);

/* Tuning: the first product call for a (precision, kernel, dimension, tile
 * count) shape times the candidate launch shapes on `stream` (about 20 products,
 * waiting for their events) and keeps the fastest for the process (and in the
 * file KRR_TUNE_CACHE names); that first call is therefore synchronous.  Calls
 * on a stream that is being captured into a HIP graph use the default shape
 * instead and never tune.  Results do not depend on the launch shape.
 *
 * y = K_hat q + shift q  (section 3.1: the weighted kernel summation, here with
 * the regularisation shift of eq. RegKernel; shift = gamma gives K, shift =
 * delta gives M).  prec KRR_FP64: q, y are double[n]; KRR_FP32 / KRR_BF16:
 * float[n].  The product is computed on the fly; K_hat is never formed.  y may
 * not alias q.  Errors: KRR_EINVAL (n < 1, d outside 1..KRR_MAX_DIM, sigma <= 0
 * or not finite, shift not finite, NULL pointers), KRR_EWORKSPACE. */
int kmvp_gauss(const krr_points *pts /* host */, double sigma, double shift, int32_t prec,
               const void *q, void *y, void *ws, size_t ws_bytes, krr_stream_t stream);

/* kmvp_gauss for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product, y = K_hat q + shift q, with the same arguments except the workspace,
 * which is a fixed static device array of krr_noalloc_scratch_bytes() bytes
 * (128 MiB) that every device the library runs on holds until the process ends.
 * Nothing is allocated or freed, no launch shape is tuned (the tuned shape of
 * an earlier kmvp_gauss call on the same shape, else the default one; the result
 * does not depend on it) and nothing is synchronised.  Every call on a device
 * shares that device's array, which keeps the last call's contents: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  Errors as kmvp_gauss, and KRR_EUNSUPPORTED when the
 * product's scratch (krr_workspace_size(KRR_WS_KMVP, ...): about 1 KB per point,
 * mostly partial-sum slots, plus 17 MiB at d = 3, so up to about 120,000 points
 * there) exceeds the array. */
size_t krr_noalloc_scratch_bytes(void);
int kmvp_gauss_noalloc(const krr_points *pts /* host */, double sigma, double shift, int32_t prec,
                       const void *q, void *y, krr_stream_t stream);

/* The same product with the Matern-3/2 kernel (eq. MaternKernel, section 6):
 * y = K_hat q + shift q, K_hat_ij = (1 + sqrt(3) d_ij) exp(-sqrt(3) d_ij),
 * d_ij = ||x_i - x_j|| / h.  Arguments, layouts and errors as in kmvp_gauss
 * (h in place of sigma, h > 0; the KRR_WS_KMVP workspace size). */
int kmvp_matern(const krr_points *pts /* host */, double h, double shift, int32_t prec,
                const void *q, void *y, void *ws, size_t ws_bytes, krr_stream_t stream);

/* Y[:, r] = K_hat Q[:, r] + shift Q[:, r] for r < nrhs (several right-hand
 * sides, the multi-RHS need of the posterior variance, section 2.1).  Q and Y are
 * column-major with leading dimensions ldq, ldy >= n; element types as in
 * kmvp_gauss.  The kernel tile is formed once per pair and applied to all
 * columns on the matrix cores. */
int kmvp_gauss_multi(const krr_points *pts /* host */, double sigma, double shift, int32_t prec,
                     int32_t nrhs, const void *Q, int64_t ldq, void *Y, int64_t ldy,
                     void *ws, size_t ws_bytes, krr_stream_t stream);

/* Rectangular product y = K_hat(targets, sources) q: y_i = sum_j k(t_i, s_j) q_j
 * for i < targets->n (the prediction k(x*)^T w of eq. GPR_mean and eq. Kriging).
 * Both point sets have the same d.  Element types as in kmvp_gauss. */
int kmvp_gauss_cross(const krr_points *targets /* host */, const krr_points *sources /* host */,
                     double sigma, int32_t prec, const void *q, void *y,
                     void *ws, size_t ws_bytes, krr_stream_t stream);

/* Adjoint pass for the gradient of a loss l(w), w = K^{-1} y (hyperparameters
 * by maximum likelihood, section 2.1).  Given lam = K^{-1} dl/dw and w, writes
 * dl/dtheta = -lam^T (dK/dtheta) w:
 *   gx[i*d + t]   = (1/sigma^2) sum_j (lam_i w_j + lam_j w_i) K_hat_ij (x_it - x_jt)
 *   *g_logsigma   = -(1/sigma^2) sum_ij lam_i w_j K_hat_ij ||x_i - x_j||^2
 *   *g_loggamma   = -gamma lam^T w
 * gx is n x d row-major double (device); g_logsigma and g_loggamma are single
 * doubles in device memory.  lam may equal w (the case l = y^T K^{-1} y).
 * prec: KRR_FP64 (kernel values, differences and sums in FP64) or KRR_FP32
 * (FP32 pair loop, FP64 epilogue); other values give KRR_EINVAL.  At the
 * solution of an ill-conditioned system the row sums cancel heavily, so the
 * FP32 pass loses accuracy well beyond FP32 rounding. */
int kmvp_grad(const krr_points *pts /* host */, double sigma, double gamma, int32_t prec,
              const double *lam, const double *w, double *gx, double *g_logsigma,
              double *g_loggamma, void *ws, size_t ws_bytes, krr_stream_t stream);

/* Truncated CG for the preconditioner system (K_hat + shift I) z = v from z = 0
 * (sections 4.3, 5.2): at most maxit iterations (>= 1), stopping early when the
 * recursive residual satisfies ||r|| / ||v|| <= tol (tol = 0: always maxit).
 * Vectors are double[n] for KRR_FP64, float[n] otherwise.  info (host, may be
 * NULL) receives the iteration count; passing it synchronises the stream. */
int cg_inner_solve(const krr_points *pts /* host */, double sigma, double shift, int32_t prec,
                   const void *v, void *z, int32_t maxit, double tol, krr_info *info /* host */,
                   void *ws, size_t ws_bytes, krr_stream_t stream);

/* Flexible GMRES (Algorithm 1) for (K_hat + gamma I) x = b, right-preconditioned
 * by inner CG solves of M = K_hat + delta I in opts->inner_prec, outer product,
 * Gram-Schmidt and Givens least squares in FP64.  b, x: double[n]; x holds the
 * initial guess on entry (warm start; zero it for x0 = 0) and the solution on
 * exit.  Convergence is declared on the true FP64 residual.  Returns KRR_OK,
 * KRR_NOT_CONVERGED (max_outer reached; best iterate in x) or an error. */
int fgmres_solve(const krr_points *pts /* host */, double sigma, double gamma, const double *b,
                 double *x, const krr_fgmres_opts *opts /* host, may be NULL */,
                 krr_info *info /* host, may be NULL */, void *ws, size_t ws_bytes,
                 krr_stream_t stream);

/* Solve nprob independent systems, each with nrhs right-hand sides:
 * (K_hat_k + gamma_k I) W_k = Y_k.  The paper solves one kriging system per week
 * of data, each on its own points (kriging experiment, section 6.3), and the GPR
 * posterior variance needs one solve with K_hat + gamma I per test point
 * (section 2.1, the variance after eq. GPR_mean): the systems share nothing but
 * the method, and every (system, column) pair is solved as in fgmres_solve.  probs, sigma, gamma, Y, W, ldy are host
 * arrays of length nprob; Y[k] and W[k] are device pointers to column-major
 * n_k x nrhs blocks with leading dimension ldy[k] >= n_k (ldy may be NULL:
 * ld = n_k).  W[k] is overwritten (x0 = 0).  mode is a krr_mode.  infos (host,
 * may be NULL) has nprob*nrhs entries, entry k*nrhs + r for column r of system k.
 * With nprob == 1 and nrhs == 1 this is fgmres_solve / the plain CG.  Several
 * systems or columns of the Gaussian kernel run together in modes FGMRES,
 * GMRES and CG64: their kernel products are batched into multi-column launches
 * (one per dimension class, its work-item tile autotuned on the first call for
 * that shape), every (system, column) pair keeps its own solver state and
 * stops on its own, each outer step of the flexible solver is one HIP graph
 * replay, and the host reads a small summary every opts->cg_check steps (the
 * mixed solve) or iterations (CG64).  FGMRES with KRR_FP64 inner products, FCG
 * and the Matern kernel solve the pairs one after the other.  A right-hand-side
 * column with a non-finite value is not solved (its W column is zero, its info
 * status KRR_ENONFINITE) while the other columns are; the call then returns
 * KRR_ENONFINITE.  A column that breaks down (non-finite or non-positive
 * curvature during the iteration) is retired with KRR_BREAKDOWN and keeps its
 * last finite iterate; the others continue.  Otherwise returns the worst status
 * over all pairs. */
int krr_solve(const krr_points *probs /* host */, int32_t nprob, const double *sigma /* host */,
              const double *gamma /* host */, int32_t nrhs, const double *const *Y /* host array */,
              const int64_t *ldy /* host, may be NULL */, double *const *W /* host array */,
              int32_t mode, const krr_fgmres_opts *opts /* host, may be NULL */,
              krr_info *infos /* host, may be NULL */, void *ws, size_t ws_bytes,
              krr_stream_t stream);

/* GPR prediction (section 2.1): at the m test points, the posterior mean
 * (eq. GPR_mean; with w = (K_hat + gamma I)^{-1} y from a solve, mean = K_hat(test,
 * train) w, also the kriging interpolant of eq. Kriging) and, when var is not
 * NULL, the posterior variance
 *   var_j = k(x*_j, x*_j) - k_j^T (K_hat + gamma I)^{-1} k_j,  k_j = K_hat(train, x*_j),
 * by multi-right-hand-side solves of the training system (16 test points per
 * batch; krr_solve with opts, mode FGMRES).  train, test: n x d and m x d
 * row-major double (device); w: double[n]; mean, var: double[m] (device).
 * opts->kernel selects the kernel (sigma: bandwidth or length scale).  infos
 * (host, may be NULL): m entries, the solve of test point j.  Workspace:
 * krr_workspace_size(KRR_WS_PREDICT, {train, test}, 2, 1, opts).  Returns the
 * worst solve status (KRR_OK when var is NULL) or an error. */
int krr_predict(const krr_points *train /* host */, const krr_points *test /* host */, double sigma,
                double gamma, const double *w, double *mean, double *var,
                const krr_fgmres_opts *opts /* host, may be NULL */, krr_info *infos /* host, may be NULL */,
                void *ws, size_t ws_bytes, krr_stream_t stream);

/* Extreme eigenvalues of the k x k Lanczos tridiagonal of a conjugate gradient
 * run (section 3: CG on a symmetric positive definite matrix is the Lanczos
 * process; the condition number bounds its convergence).  alpha[j] is the j-th
 * step length and beta[j] = r_{j+1}.r_{j+1} / r_j.r_j (j = 0 .. k-1; beta[k-1] is
 * not used).  The tridiagonal has diagonal 1/alpha_0 and
 * 1/alpha_j + beta_{j-1}/alpha_{j-1} (j >= 1) and off-diagonal
 * sqrt(beta_{j-1})/alpha_{j-1}; its extreme eigenvalues are found by Sturm-count
 * bisection to about 1e-15 relative.  Host arrays; host computation only (no
 * device call).  Returns KRR_OK, or KRR_EINVAL for null pointers, k < 1, or a
 * non-finite or non-positive alpha or negative beta. */
int krr_lanczos_extremes(const double *alpha /* host, k */, const double *beta /* host, k */, int32_t k,
                         double *lambda_min /* host */, double *lambda_max /* host */);

/* Launch timing of the kernel products (measurement support).  Between
 * krr_profile_begin() and krr_profile_end() every kernel-product launch made by
 * any call on this process records a pair of HIP events on its own stream
 * around the product kernel (the main O(N^2) kernel, not the O(N) partial-sum
 * kernel).  krr_profile_end() waits for the recorded events and returns, per
 * product precision, the launch count, the summed kernel time and the summed
 * algorithmic pair count (n_targets x n_sources, padding excluded), of which
 * pairs_skipped were in far tile pairs (exactly zero, not evaluated).  At most
 * max_launches launches are recorded (later ones are counted in `dropped`).
 * No device memory is allocated (the skipped-pair counters are a static device
 * array); begin and end synchronise the device.  Not thread-safe. */
typedef struct {
    int64_t launches;
    double total_ms;
    double pairs;
    double pairs_skipped; /* of `pairs`, those in tile pairs the product kernels skipped because every
                             kernel value there is exactly zero in the product's precision (far tiles) */
} krr_profile_entry;

typedef struct {
    krr_profile_entry prec[3]; /* indexed by krr_prec */
    int64_t dropped;
} krr_profile_stats;

int krr_profile_begin(int32_t max_launches);
int krr_profile_end(krr_profile_stats *out /* host */);

/* Issue-rate probe (measurement support, not part of the method): times six
 * register-only kernels on `stream` and writes rates[0] = FP32 FMA lane-ops/s,
 * rates[1] = exp2 + dependent FMA pairs/s, rates[2] = 16x16x4 FP32 matrix-core
 * pairs/s (4 multiply-adds per pair), rates[3] = pairs/s of the FP32
 * matrix-core exponent product's instruction mix (per 1024 pairs: four 16x16x4
 * FP32 matrix-core operations, 16 exp2 and 16 FMAs per lane), rates[4] = pairs/s
 * of the split-f16 product's mix (per 1024 pairs: one 32x32x16 f16 matrix-core
 * operation, 16 exp2 and 16 FMAs per lane), rates[5] = FP64 exp2 + dependent
 * FP64 FMA pairs/s (the FP64 products' per-pair VALU work).  rates: host array
 * of 6 doubles.
 * ws: device workspace of at least krr_probe_workspace_size() bytes (scratch,
 * overwritten).  Synchronises the stream.  Returns KRR_OK, KRR_EINVAL,
 * KRR_EWORKSPACE or KRR_EHIP. */
size_t krr_probe_workspace_size(void);
int krr_probe_issue_rates(double *rates /* host, 6 */, void *ws, size_t ws_bytes, krr_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* KRR_H */
