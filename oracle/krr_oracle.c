/*
 * krr_oracle.c -- plain, slow, double-precision CPU oracle for the
 * flexible-preconditioned Krylov solution of regularised Gaussian kernel
 * systems (Srinivasan, Hu, Gumerov, Murtugudde, Duraiswami, "Preconditioned
 * Krylov solvers for kernel regression").
 *
 * TEST INFRASTRUCTURE.  This file is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the GPU library never links, calls or includes
 * it, and it shares no code with the GPU library.
 *
 * Every routine is written straight from its definition, in FP64, with libm
 * exp and plain loops in index order; no blocking, fusion or reordering.  The
 * only parallelism is an OpenMP split over output rows of the kernel sums,
 * which leaves each row's summation order unchanged (results do not depend on
 * the thread count).
 *
 * Notation follows the paper: X = {x_1..x_N} in R^d, K_hat_ij = k(x_i, x_j)
 * (eq. kernelMatrix, section 1) with the Gaussian k (eq. Gaussian, section 1),
 * K = K_hat + gamma I (eq. RegKernel), preconditioner M = K_hat + delta I
 * (section 5, the proposed preconditioner).  The Matern kernel of section 6
 * (eq. MaternKernel) has its own kernel sums (or_matern_*).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Gaussian kernel, eq. (Gaussian), section 1:
 *   Phi(a, b) = exp(-||a - b||^2 / (2 sigma^2)). */
double or_gauss(const double *a, const double *b, int d, double sigma)
{
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = a[t] - b[t];
        r2 += diff * diff;
    }
    return exp(-r2 / (2.0 * sigma * sigma));
}

/* Explicit kernel matrix, eq. (kernelMatrix), section 1, including the
 * diagonal k(x_i, x_i).  K is nt x ns row-major: K[i*ns + j] = k(xt_i, xs_j).
 * Points are row-major (one point of d coordinates per row). */
void or_kernel_matrix(int64_t nt, int64_t ns, int d, const double *xt,
                      const double *xs, double sigma, double *K)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; ++i)
        for (int64_t j = 0; j < ns; ++j)
            K[i * ns + j] = or_gauss(xt + i * d, xs + j * d, d, sigma);
}

/* Weighted kernel summation computed on the fly (section 1 and section 3.1,
 * "Fast matrix-vector products"): y_i = sum_j k(xt_i, xs_j) q_j.  When the
 * target and source sets are the same point set (nt == ns and xt == xs) the
 * shift term shift * q_i is added, giving y = (K_hat + shift I) q; a
 * rectangular product has no shift term (shift is ignored there). */
void or_mvp(int64_t nt, int64_t ns, int d, const double *xt, const double *xs,
            double sigma, double shift, const double *q, double *y)
{
    const int square = (nt == ns && xt == xs);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < ns; ++j)
            acc += or_gauss(xt + i * d, xs + j * d, d, sigma) * q[j];
        y[i] = square ? acc + shift * q[i] : acc;
    }
}

/* The same sum for a subset of rows: y_rows[k] = ((K_hat + shift I) q)_{rows[k]}.
 * Used to check large products on sampled rows. */
void or_mvp_rows(int64_t n, int d, const double *x, double sigma, double shift,
                 const double *q, int64_t nrows, const int64_t *rows, double *y_rows)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j)
            acc += or_gauss(x + i * d, x + j * d, d, sigma) * q[j];
        y_rows[k] = acc + shift * q[i];
    }
}

/* Several right-hand sides: Y[:, r] = (K_hat + shift I) Q[:, r], with column
 * r of Q at Q + r*ldq and of Y at Y + r*ldy (column-major blocks). */
void or_mvp_multi(int64_t n, int d, const double *x, double sigma, double shift,
                  int nrhs, const double *Q, int64_t ldq, double *Y, int64_t ldy)
{
    for (int r = 0; r < nrhs; ++r)
        or_mvp(n, n, d, x, x, sigma, shift, Q + r * ldq, Y + r * ldy);
}

/* Matern kernel with smoothness 3/2, eq. (MaternKernel), section 6 (the
 * non-Gaussian kernel of Table 2):
 *   k(a, b) = (1 + sqrt(3) r) exp(-sqrt(3) r),  r = ||a - b|| / h. */
double or_matern(const double *a, const double *b, int d, double h)
{
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = a[t] - b[t];
        r2 += diff * diff;
    }
    double s = sqrt(3.0) * sqrt(r2) / h;
    return (1.0 + s) * exp(-s);
}

/* Explicit Matern kernel matrix (eq. kernelMatrix with eq. MaternKernel),
 * K[i*ns + j] = k(xt_i, xs_j). */
void or_matern_matrix(int64_t nt, int64_t ns, int d, const double *xt,
                      const double *xs, double h, double *K)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; ++i)
        for (int64_t j = 0; j < ns; ++j)
            K[i * ns + j] = or_matern(xt + i * d, xs + j * d, d, h);
}

/* On-the-fly Matern sum y_i = sum_j k(xt_i, xs_j) q_j (+ shift q_i when the
 * two point sets are the same set, as in or_mvp). */
void or_matern_mvp(int64_t nt, int64_t ns, int d, const double *xt, const double *xs,
                   double h, double shift, const double *q, double *y)
{
    const int square = (nt == ns && xt == xs);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < ns; ++j)
            acc += or_matern(xt + i * d, xs + j * d, d, h) * q[j];
        y[i] = square ? acc + shift * q[i] : acc;
    }
}

/* ((K_hat + shift I) q)_{rows[k]} with the Matern kernel. */
void or_matern_mvp_rows(int64_t n, int d, const double *x, double h, double shift,
                        const double *q, int64_t nrows, const int64_t *rows, double *y_rows)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j)
            acc += or_matern(x + i * d, x + j * d, d, h) * q[j];
        y_rows[k] = acc + shift * q[i];
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(int64_t n, const double *a)
{
    return sqrt(dot(n, a, a));
}

/* Direct solve (the "Direct" column of Table 1, section 6.1): textbook
 * Cholesky A = L L^T computed in place in the lower triangle of the n x n
 * row-major A (the strict upper triangle is zeroed).  Returns 0, or -(k+1) when
 * the k-th pivot is not positive. */
int or_cholesky(int64_t n, double *A)
{
    for (int64_t j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return (int)(-(j + 1));
        double ljj = sqrt(s);
        A[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / ljj;
        }
        for (int64_t i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return 0;
}

/* Forward then back substitution with the factor from or_cholesky:
 * x = (L L^T)^{-1} b. */
void or_chol_solve(int64_t n, const double *L, const double *b, double *x)
{
    double *z = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * z[k];
        z[i] = s / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
    free(z);
}

/* Conjugate gradient on (K_hat + shift I) w = b (section 3: CG is the Krylov
 * method for symmetric positive definite kernel matrices; it is the paper's
 * unpreconditioned solver and its inner solver).  Hestenes-Stiefel form with
 * w0 = 0:
 *   r = b, p = r; repeat: alpha = r.r / p.Ap, w += alpha p, r -= alpha Ap,
 *   beta = r_new.r_new / r.r, p = r + beta p.
 * Two stopping modes:
 *   confirm = 0 (the inner preconditioner solve, section 4.3 / 5.2): stop after
 *     maxit iterations or when ||r|| / ||b|| <= tol on the recursive residual,
 *     or when r is exactly zero;
 *   confirm = 1 (the plain solver): when the recursive residual reaches tol the
 *     true residual b - (K_hat + shift I) w is computed; if it is above tol the
 *     iteration restarts from w with r = p = the true residual.
 * Returns 0 when converged (confirm = 1) or when the loop ended (confirm = 0),
 * 1 when maxit was reached without convergence in confirm mode, and 2 on a
 * breakdown (p.Ap <= 0 or not finite).  *iters receives the iteration count;
 * *relres the final relative residual (true when confirm = 1, recursive
 * otherwise); hist (length >= maxit + 1, may be NULL) the recursive relative
 * residual before each iteration and after the last. */
int or_cg(int64_t n, int d, const double *x, double sigma, double shift,
          const double *b, double *w, int maxit, double tol, int confirm,
          int *iters, double *relres, double *hist)
{
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *p = (double *)malloc((size_t)n * sizeof(double));
    double *Ap = (double *)malloc((size_t)n * sizeof(double));
    double bn = nrm2(n, b);
    int status = 1, it = 0;
    for (int64_t i = 0; i < n; ++i) { w[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    double rr = dot(n, r, r);
    double rel = (bn > 0.0) ? sqrt(rr) / bn : 0.0;
    if (hist) hist[0] = rel;
    if (bn == 0.0) { status = 0; goto done; }
    while (it < maxit) {
        if (rr == 0.0) { status = 0; break; }
        if (rel <= tol) {
            if (!confirm) { status = 0; break; }
            or_mvp(n, n, d, x, x, sigma, shift, w, Ap);
            for (int64_t i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
            rr = dot(n, r, r);
            rel = sqrt(rr) / bn;
            if (rel <= tol) { status = 0; break; }
            for (int64_t i = 0; i < n; ++i) p[i] = r[i];
        }
        or_mvp(n, n, d, x, x, sigma, shift, p, Ap);
        double pAp = dot(n, p, Ap);
        if (!(pAp > 0.0) || !isfinite(pAp)) { status = 2; break; }
        double alpha = rr / pAp;
        for (int64_t i = 0; i < n; ++i) { w[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rr_new = dot(n, r, r);
        double beta = rr_new / rr;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        rel = sqrt(rr) / bn;
        ++it;
        if (hist) hist[it] = rel;
    }
    if (status == 1 && !confirm) status = 0;
    if (status == 1 && confirm && rel <= tol) {
        or_mvp(n, n, d, x, x, sigma, shift, w, Ap);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
        rel = nrm2(n, r) / bn;
        if (rel <= tol) status = 0;
    }
done:
    *iters = it;
    *relres = rel;
    free(r); free(p); free(Ap);
    return status;
}

/* Flexible GMRES (Algorithm 1, section 4.2) for K w = b, K = K_hat + gamma I,
 * read with 1-based indices as in Saad's FGMRES(m):
 *
 *   r0 = b - K x0, beta = ||r0||, v_1 = r0 / beta
 *   for j = 1..m:
 *     z_j  = inner preconditioner solve M z = v_j              (inner Krylov)
 *     w    = K z_j
 *     for i = 1..j:  h_ij = (w, v_i);  w = w - h_ij v_i      (modified Gram-Schmidt)
 *     h_{j+1,j} = ||w||,  v_{j+1} = w / h_{j+1,j}
 *   y = argmin || beta e_1 - H_bar y ||,  x = x0 + Z y;  restart from x if needed.
 *
 * The least-squares problem is solved with Givens rotations applied column by
 * column (the standard way of keeping its residual |g_{j+1}| current after every
 * step).  A cycle ends early when |g_{j+1}| / ||b|| <= tol or on a "happy"
 * breakdown, h_{j+1,j} <= 1e-14 ||w before orthogonalisation|| (then the Krylov
 * space is invariant and the least-squares solution is exact).  After each
 * cycle the true residual b - K x is recomputed; the solve stops when its
 * relative norm is <= tol, otherwise it restarts.
 *
 * Inner preconditioner (section 4.3 and section 5):
 *   inner_mode 0: z_j = v_j (M = I: plain GMRES, the unpreconditioned variant);
 *   inner_mode 1: z_j = CG on (K_hat + delta I) z = v_j from z = 0, stopped after
 *                 inner_maxit iterations or at recursive relative residual
 *                 <= inner_tol (truncated inner CG, section 5.2).
 *
 * Parameters: m restart length, max_outer cap on the total number of outer
 * steps (all cycles).  x holds x0 on entry and the solution on exit.
 * Outputs (any may be NULL): info[0] total outer steps, info[1] total inner CG
 * iterations, info[2] number of cycles, info[3] 1 if a happy breakdown ended a
 * cycle; est_hist[k] (length >= max_outer) the estimate |g_{j+1}| / ||b|| after
 * outer step k; true_hist[c] (length >= max_outer) the true relative residual
 * after cycle c; *relres the final true relative residual.  When V_out, Z_out,
 * H_out are given they receive the last cycle's basis V (n x (m+1), column j at
 * V_out + j*n), directions Z (n x m) and Hessenberg H_bar ((m+1) x m,
 * row-major, entry (i, j) at H_out[i*m + j], before rotation) and *k_out the
 * number of steps in that cycle.
 * Returns 0 converged, 1 not converged within max_outer. */
int or_fgmres(int64_t n, int d, const double *x_pts, double sigma, double gamma,
              const double *b, double *x, int m, int max_outer, double tol,
              int inner_mode, double delta, int inner_maxit, double inner_tol,
              int *info, double *est_hist, double *true_hist, double *relres,
              double *V_out, double *Z_out, double *H_out, int *k_out)
{
    double *V = (double *)calloc((size_t)n * (m + 1), sizeof(double));
    double *Z = (double *)calloc((size_t)n * m, sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));   /* rotated copy */
    double *Hraw = (double *)calloc((size_t)(m + 1) * m, sizeof(double)); /* as built */
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *yv = (double *)calloc((size_t)m, sizeof(double));
    double *wv = (double *)malloc((size_t)n * sizeof(double));
    double *tmp = (double *)malloc((size_t)n * sizeof(double));
    double bn = nrm2(n, b);
    int outer = 0, inner_total = 0, cycles = 0, happy = 0, status = 1, kcyc = 0;
    double rel = 0.0;

    if (bn == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = 0;
        goto done;
    }
    for (;;) {
        /* r0 = b - K x0, beta = ||r0||, v_1 = r0 / beta */
        or_mvp(n, n, d, x_pts, x_pts, sigma, gamma, x, tmp);
        for (int64_t i = 0; i < n; ++i) wv[i] = b[i] - tmp[i];
        double beta = nrm2(n, wv);
        rel = beta / bn;
        if (cycles > 0 && true_hist) true_hist[cycles - 1] = rel;
        if (rel <= tol) { status = 0; break; }
        if (outer >= max_outer) { status = 1; break; }
        for (int64_t i = 0; i < n; ++i) V[i] = wv[i] / beta;
        memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
        memset(Hraw, 0, sizeof(double) * (size_t)(m + 1) * m);
        memset(g, 0, sizeof(double) * (size_t)(m + 1));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && outer < max_outer; ++j) {
            double *vj = V + (int64_t)j * n;
            double *zj = Z + (int64_t)j * n;
            /* inner preconditioner: M_j z_j = v_j */
            if (inner_mode == 0) {
                for (int64_t i = 0; i < n; ++i) zj[i] = vj[i];
            } else {
                int it_in = 0;
                double rr_in = 0.0;
                or_cg(n, d, x_pts, sigma, delta, vj, zj, inner_maxit, inner_tol, 0,
                      &it_in, &rr_in, NULL);
                inner_total += it_in;
            }
            /* w = K z_j */
            or_mvp(n, n, d, x_pts, x_pts, sigma, gamma, zj, wv);
            double wnorm0 = nrm2(n, wv);
            /* modified Gram-Schmidt */
            for (int i = 0; i <= j; ++i) {
                double *vi = V + (int64_t)i * n;
                double hij = dot(n, wv, vi);
                H[i * m + j] = hij;
                Hraw[i * m + j] = hij;
                for (int64_t t = 0; t < n; ++t) wv[t] -= hij * vi[t];
            }
            double hnext = nrm2(n, wv);
            H[(j + 1) * m + j] = hnext;
            Hraw[(j + 1) * m + j] = hnext;
            int breakdown = !(hnext > 1e-14 * wnorm0);
            if (!breakdown) {
                double *vn = V + (int64_t)(j + 1) * n;
                for (int64_t t = 0; t < n; ++t) vn[t] = wv[t] / hnext;
            }
            /* apply the previous rotations to column j, then a new one */
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            {
                double a = H[j * m + j], c = H[(j + 1) * m + j];
                double rho = sqrt(a * a + c * c);
                cs[j] = a / rho;
                sn[j] = c / rho;
                H[j * m + j] = rho;
                H[(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
            }
            ++outer;
            k = j + 1;
            if (est_hist) est_hist[outer - 1] = fabs(g[j + 1]) / bn;
            if (breakdown) { happy = 1; break; }
            if (fabs(g[j + 1]) / bn <= tol) break;
        }
        /* y = R^{-1} g (back substitution), x = x0 + Z y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t < k; ++t) s -= H[i * m + t] * yv[t];
            yv[i] = s / H[i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (int64_t t = 0; t < n; ++t) x[t] += yv[i] * Z[(int64_t)i * n + t];
        ++cycles;
        kcyc = k;
        if (V_out) memcpy(V_out, V, sizeof(double) * (size_t)n * (m + 1));
        if (Z_out) memcpy(Z_out, Z, sizeof(double) * (size_t)n * m);
        if (H_out) memcpy(H_out, Hraw, sizeof(double) * (size_t)(m + 1) * m);
    }
done:
    if (info) { info[0] = outer; info[1] = inner_total; info[2] = cycles; info[3] = happy; }
    if (relres) *relres = rel;
    if (k_out) *k_out = kcyc;
    free(V); free(Z); free(H); free(Hraw); free(cs); free(sn); free(g); free(yv);
    free(wv); free(tmp);
    return status;
}

/* Flexible CG for K w = b, K = K_hat + gamma I, from w = 0: the flexible
 * Krylov alternative to Algorithm 1 that section 4.2 and section 5.4 compare
 * it with.  With a preconditioner that changes from step to step, the new
 * search direction is made K-orthogonal to the previous ones explicitly (the
 * re-orthogonalisation the paper attributes to Notay); at most mmax previous
 * directions are kept:
 *   r_0 = b
 *   for i = 0, 1, ...:
 *     z_i = inner preconditioner solve M z = r_i       (as in or_fgmres)
 *     d_i = z_i - sum_{k in window} ((z_i . q_k) / (d_k . q_k)) d_k,  q_k = K d_k
 *     q_i = K d_i
 *     alpha_i = (d_i . r_i) / (d_i . q_i)
 *     w += alpha_i d_i,   r_{i+1} = r_i - alpha_i q_i
 * the window being the last min(i, mmax) directions.  When the recursive
 * residual reaches ||r|| / ||b|| <= tol the true residual b - K w is computed;
 * above tol the iteration restarts from it with an empty window.
 * Outputs: info[0] outer iterations, info[1] inner CG iterations;
 * hist (length >= max_outer + 1, may be NULL) the recursive relative residual
 * before each iteration and after the last; D_out (n x max_outer, may be NULL)
 * the directions d_i of the last restart, column i at D_out + i*n; *relres the
 * final true relative residual.  Returns 0 converged, 1 not converged within
 * max_outer, 2 on a breakdown (d.q <= 0 or not finite). */
int or_fcg(int64_t n, int d, const double *x_pts, double sigma, double gamma,
           const double *b, double *w, int mmax, int max_outer, double tol,
           int inner_mode, double delta, int inner_maxit, double inner_tol,
           int *info, double *hist, double *D_out, double *relres)
{
    if (mmax < 1) mmax = 1;
    double *D = (double *)calloc((size_t)n * mmax, sizeof(double));
    double *Q = (double *)calloc((size_t)n * mmax, sizeof(double));
    double *dq = (double *)calloc((size_t)mmax, sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double bn = nrm2(n, b);
    int it = 0, inner_total = 0, status = 1, cnt = 0, head = 0, restart_i = 0;
    double rel = 0.0;
    for (int64_t i = 0; i < n; ++i) { w[i] = 0.0; r[i] = b[i]; }
    if (bn == 0.0) { status = 0; goto done; }
    rel = nrm2(n, r) / bn;
    if (hist) hist[0] = rel;
    while (it < max_outer) {
        if (rel <= tol) {
            /* confirm with the true residual; restart from it if needed */
            or_mvp(n, n, d, x_pts, x_pts, sigma, gamma, w, q);
            for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
            rel = nrm2(n, r) / bn;
            if (rel <= tol) { status = 0; break; }
            cnt = 0;
            head = 0;
            restart_i = it;
        }
        if (inner_mode == 0) {
            for (int64_t i = 0; i < n; ++i) z[i] = r[i];
        } else {
            int it_in = 0;
            double rr_in = 0.0;
            or_cg(n, d, x_pts, sigma, delta, r, z, inner_maxit, inner_tol, 0, &it_in, &rr_in, NULL);
            inner_total += it_in;
        }
        /* d = z - sum_k (z.q_k / d_k.q_k) d_k over the window (oldest first) */
        double *dn = D + (int64_t)head * n;
        double *qn = Q + (int64_t)head * n;
        for (int64_t i = 0; i < n; ++i) q[i] = z[i];
        for (int c = cnt; c >= 1; --c) {
            int k = (head - c + mmax) % mmax;
            double beta = dot(n, z, Q + (int64_t)k * n) / dq[k];
            for (int64_t i = 0; i < n; ++i) q[i] -= beta * D[(int64_t)k * n + i];
        }
        for (int64_t i = 0; i < n; ++i) dn[i] = q[i];
        or_mvp(n, n, d, x_pts, x_pts, sigma, gamma, dn, qn);
        double dqi = dot(n, dn, qn);
        if (!(dqi > 0.0) || !isfinite(dqi)) { status = 2; break; }
        dq[head] = dqi;
        double alpha = dot(n, dn, r) / dqi;
        for (int64_t i = 0; i < n; ++i) { w[i] += alpha * dn[i]; r[i] -= alpha * qn[i]; }
        if (D_out && it - restart_i < max_outer)
            memcpy(D_out + (int64_t)(it - restart_i) * n, dn, sizeof(double) * (size_t)n);
        head = (head + 1) % mmax;
        if (cnt < mmax) ++cnt;
        ++it;
        rel = nrm2(n, r) / bn;
        if (hist) hist[it] = rel;
    }
    if (status == 1 && rel <= tol) {
        or_mvp(n, n, d, x_pts, x_pts, sigma, gamma, w, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        rel = nrm2(n, r) / bn;
        if (rel <= tol) status = 0;
    }
done:
    if (info) { info[0] = it; info[1] = inner_total; }
    if (relres) *relres = rel;
    free(D); free(Q); free(dq); free(r); free(z); free(q);
    return status;
}

/* GPR prediction (section 2.1): posterior mean (eq. GPR_mean) and variance
 * (the equation after it) at m test points xs from n training points x,
 *   mean_j = k_j^T (K_hat + gamma I)^{-1} y,
 *   var_j  = k(xs_j, xs_j) - k_j^T (K_hat + gamma I)^{-1} k_j,
 * k_j = [k(x_1, xs_j), ..., k(x_n, xs_j)]^T, with the explicit matrix and the
 * textbook Cholesky solve.  kernel 0: Gaussian (sigma), 1: Matern-3/2 (length
 * scale sigma).  var may be NULL.  Returns 0, or -1 if the matrix is not
 * positive definite. */
int or_predict(int64_t n, int64_t m, int d, const double *x, const double *xs, double sigma,
               double gamma, int kernel, const double *y, double *mean, double *var)
{
    double *K = (double *)malloc((size_t)n * n * sizeof(double));
    double *Ks = (double *)malloc((size_t)n * m * sizeof(double));   /* K_hat(x, xs), n x m */
    double *a = (double *)malloc((size_t)n * sizeof(double));
    double *col = (double *)malloc((size_t)n * sizeof(double));
    double *sol = (double *)malloc((size_t)n * sizeof(double));
    int rc = 0;
    if (kernel == 1) {
        or_matern_matrix(n, n, d, x, x, sigma, K);
        or_matern_matrix(n, m, d, x, xs, sigma, Ks);
    } else {
        or_kernel_matrix(n, n, d, x, x, sigma, K);
        or_kernel_matrix(n, m, d, x, xs, sigma, Ks);
    }
    for (int64_t i = 0; i < n; ++i) K[i * n + i] += gamma;
    if (or_cholesky(n, K) != 0) { rc = -1; goto done; }
    or_chol_solve(n, K, y, a);                       /* a = (K_hat + gamma I)^{-1} y */
    for (int64_t j = 0; j < m; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += Ks[i * m + j] * a[i];
        mean[j] = s;
        if (var) {
            for (int64_t i = 0; i < n; ++i) col[i] = Ks[i * m + j];
            or_chol_solve(n, K, col, sol);
            double kk = (kernel == 1) ? or_matern(xs + j * d, xs + j * d, d, sigma)
                                      : or_gauss(xs + j * d, xs + j * d, d, sigma);
            double t = 0.0;
            for (int64_t i = 0; i < n; ++i) t += col[i] * sol[i];
            var[j] = kk - t;
        }
    }
done:
    free(K); free(Ks); free(a); free(col); free(sol);
    return rc;
}

/* Gradient of a scalar loss l(w), w = K^{-1} y, with respect to the points,
 * log sigma and log gamma (hyperparameters are set by maximum likelihood,
 * section 2.1 and section 6.1).  With lambda = K^{-1} (dl/dw), matrix calculus
 * (d K^{-1} = -K^{-1} dK K^{-1}) gives dl/dtheta = -lambda^T (dK/dtheta) w.
 * Written out from dK_hat_ij / dx_it = -K_hat_ij (x_it - x_jt) / sigma^2 (for
 * both the row-i and the column-i occurrence of x_i),
 * dK_hat_ij / dlog sigma = K_hat_ij ||x_i - x_j||^2 / sigma^2 and
 * dK / dlog gamma = gamma I:
 *   gx[i*d + t] = (1/sigma^2) sum_j (lam_i w_j + lam_j w_i) K_hat_ij (x_it - x_jt)
 *   g_logsigma  = -(1/sigma^2) sum_ij lam_i w_j K_hat_ij ||x_i - x_j||^2
 *   g_loggamma  = -gamma sum_i lam_i w_i
 * For l = y^T K^{-1} y one has dl/dw = y, so lambda = w. */
void or_grad(int64_t n, int d, const double *x, double sigma, double gamma,
             const double *lam, const double *w, double *gx, double *g_logsigma,
             double *g_loggamma)
{
    double s2 = sigma * sigma;
    double *rows = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int t = 0; t < d; ++t) gx[i * d + t] = 0.0;
        double rowsum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double r2 = 0.0;
            for (int t = 0; t < d; ++t) {
                double diff = x[i * d + t] - x[j * d + t];
                r2 += diff * diff;
            }
            double k = exp(-r2 / (2.0 * s2));
            double c = (lam[i] * w[j] + lam[j] * w[i]) * k / s2;
            for (int t = 0; t < d; ++t) gx[i * d + t] += c * (x[i * d + t] - x[j * d + t]);
            rowsum += lam[i] * w[j] * k * r2;
        }
        rows[i] = rowsum;
    }
    double gs = 0.0;
    for (int64_t i = 0; i < n; ++i) gs += rows[i];
    free(rows);
    *g_logsigma = -gs / s2;
    *g_loggamma = -gamma * dot(n, lam, w);
}

/* The point gradient of or_grad for a subset of rows only:
 * gx_rows[k*d + t] = (1/sigma^2) sum_j (lam_i w_j + lam_j w_i) K_hat_ij (x_it - x_jt),
 * i = rows[k].  Used to check large gradients on sampled rows. */
void or_grad_rows(int64_t n, int d, const double *x, double sigma, const double *lam,
                  const double *w, int64_t nrows, const int64_t *rows, double *gx_rows)
{
    double s2 = sigma * sigma;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        for (int t = 0; t < d; ++t) gx_rows[k * d + t] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double r2 = 0.0;
            for (int t = 0; t < d; ++t) {
                double diff = x[i * d + t] - x[j * d + t];
                r2 += diff * diff;
            }
            double kv = exp(-r2 / (2.0 * s2));
            double c = (lam[i] * w[j] + lam[j] * w[i]) * kv / s2;
            for (int t = 0; t < d; ++t) gx_rows[k * d + t] += c * (x[i * d + t] - x[j * d + t]);
        }
    }
}
