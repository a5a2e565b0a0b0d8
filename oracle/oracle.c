/*
 * CPU oracle for the differentiable sparse Krylov solve -- TEST
 * INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never
 * does.  It shares no code, header or constant with the GPU library.
 *
 * Plain, sequential, IEEE binary64 code (built with -ffp-contract=off so no
 * fused multiply-add changes a rounding).  Every loop runs in index order;
 * every inner product is a left-to-right sum.  Nothing here is blocked,
 * fused or reordered beyond what the definitions state.
 *
 * Sources (section / equation / algorithm of arXiv 2601.13994 unless noted):
 *   orc_spmv          y = A x on CSR; the local product of the distributed
 *                     SpMV (Sec. "Distributed", Eq. forward_spmv) with one
 *                     process.
 *   orc_cg            Conjugate gradient (Hestenes-Stiefel), the recurrence of
 *                     Algorithm "Distributed CG" with P = 1 (all_reduce is the
 *                     local sum), optionally with the Jacobi preconditioner
 *                     z = D^{-1} r used by the paper's PyTorch-native backend
 *                     (Sec. "Scalability", Table tab:benchmark).
 *   orc_bicgstab      BiCGStab of van der Vorst (1992), cited by the paper
 *                     for nonsymmetric systems (Introduction, Sec. "Five
 *                     backends"); right Jacobi preconditioning; the paper
 *                     gives no steps, so the textbook preconditioned form is
 *                     used (one restart with r_hat = r on breakdown).
 *   orc_transpose     CSR transpose by counting sort (stable in row order).
 *   orc_adjoint_grad  Eq. adjoint_linear: dL/db = lambda,
 *                     dL/dA_ij = -lambda_i x_j on the sparsity pattern.
 *   orc_dense_*       dense Cholesky / LU with partial pivoting (tiny n).
 *   orc_fsai          classical factorized sparse approximate inverse
 *                     (Kolotilina & Yeremin 1993) on A's lower pattern; not in
 *                     the paper, which names learned preconditioners only as
 *                     future work.
 *   orc_probe_loss    ||G A G^T z - z||^2 and its gradient w.r.t. G's values.
 *
 * Threads (orc_set_threads, default 1).  With one thread everything above
 * holds as stated.  With T > 1 threads (OpenMP, for timing the oracle on all
 * host cores and for solving grid-size systems in the tests) the SpMV rows
 * and the element-wise vector loops of CG and BiCGStab are split over the
 * threads, which changes no result, and every inner product and residual
 * norm is the sum, in thread order, of T left-to-right partial sums over
 * contiguous index ranges of equal size: deterministic for a given T, equal
 * to the one-thread result up to the rounding of that summation order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status codes returned by the solvers */
enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2, ORC_NONFINITE = 3, ORC_BAD_INPUT = 4 };
enum { ORC_PRECOND_NONE = 0, ORC_PRECOND_JACOBI = 1 };

enum { ORC_MAX_THREADS = 256 };
static int g_threads = 1;

/* Number of threads of the parallel mode (1 = plain sequential code). */
void orc_set_threads(int threads)
{
    g_threads = threads < 1 ? 1 : threads > ORC_MAX_THREADS ? ORC_MAX_THREADS : threads;
}

/* an element-wise loop split over the threads when more than one is set */
#define PAR_FOR _Pragma("omp parallel for num_threads(g_threads) schedule(static) if(g_threads > 1)")

/* ------------------------------------------------------------------------ */
/* basic vector operations                                                   */
/* ------------------------------------------------------------------------ */

void orc_spmv(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *x, double *y)
{
    PAR_FOR
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

double orc_dot(int64_t n, const double *a, const double *b)
{
    if (g_threads > 1) {
        /* T partial sums over [n t / T, n (t+1) / T), added in t order */
        const int T = g_threads;
        double part[ORC_MAX_THREADS];
        #pragma omp parallel for num_threads(T) schedule(static, 1)
        for (int t = 0; t < T; ++t) {
            double s = 0.0;
            for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i)
                s += a[i] * b[i];
            part[t] = s;
        }
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += part[t];
        return s;
    }
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

static double nrm2(int64_t n, const double *a) { return sqrt(orc_dot(n, a, a)); }

/* Inverse of the stored diagonal; returns 0 on success, -1 when a row has no
 * stored diagonal or a zero one (Jacobi is then undefined). */
int orc_jacobi_inverse(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                       double *dinv)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        int found = 0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] == i) { d = val[k]; found = 1; }
        if (!found || d == 0.0) return -1;
        dinv[i] = 1.0 / d;
    }
    return 0;
}

/* ||b - A x||_2 */
static double residual_sq(int32_t lo, int32_t hi, const int32_t *rp, const int32_t *col,
                          const double *val, const double *b, const double *x)
{
    double s = 0.0;
    for (int32_t i = lo; i < hi; ++i) {
        double ax = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            ax += val[k] * x[col[k]];
        double r = b[i] - ax;
        s += r * r;
    }
    return s;
}

double orc_residual_norm(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                         const double *b, const double *x)
{
    if (g_threads > 1) {
        const int T = g_threads;
        double part[ORC_MAX_THREADS];
        #pragma omp parallel for num_threads(T) schedule(static, 1)
        for (int t = 0; t < T; ++t)
            part[t] = residual_sq((int32_t)((int64_t)n * t / T), (int32_t)((int64_t)n * (t + 1) / T),
                                  rp, col, val, b, x);
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += part[t];
        return sqrt(s);
    }
    return sqrt(residual_sq(0, n, rp, col, val, b, x));
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient / Jacobi-PCG                                           */
/* ------------------------------------------------------------------------ */
/*
 * x <- x0 (use_x0) or 0; r = b - A x; z = M^{-1} r; p = z; rho = r.z
 * repeat: q = A p; sigma = p.q (sigma <= 0: breakdown); alpha = rho / sigma;
 *         x += alpha p; r -= alpha q; stop when ||r|| <= max(rtol ||b||, atol);
 *         z = M^{-1} r; rho' = r.z; beta = rho'/rho; p = z + beta p.
 * The stop test uses the recursive residual's 2-norm after each r update.
 * ``alphas``/``betas`` (nullable, length max_iter) receive the coefficients
 * for Lanczos (Ritz-value) checks.  ``max_iter_run`` bounds the iterations
 * actually run (for timing samples) without changing the definition.
 */
int orc_cg(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
           const double *b, double *x, int precond, int use_x0, double rtol, double atol,
           int64_t max_iter, int64_t *iters_out, double *relres_out,
           double *alphas, double *betas)
{
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    double *dinv = malloc(sizeof(double) * (size_t)n);
    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    double bnorm = nrm2(n, b);
    double rnorm;

    if (precond == ORC_PRECOND_JACOBI && orc_jacobi_inverse(n, rp, col, val, dinv) != 0) {
        status = ORC_BAD_INPUT;
        goto done;
    }
    if (!use_x0) {
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    }
    orc_spmv(n, rp, col, val, x, q);
    PAR_FOR
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double tol = rtol * bnorm;
    if (atol > tol) tol = atol;
    rnorm = nrm2(n, r);
    if (!isfinite(rnorm) || !isfinite(bnorm)) { status = ORC_NONFINITE; goto done; }
    if (rnorm <= tol) { status = ORC_OK; goto done; }
    PAR_FOR
    for (int32_t i = 0; i < n; ++i) z[i] = precond == ORC_PRECOND_JACOBI ? dinv[i] * r[i] : r[i];
    PAR_FOR
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = orc_dot(n, r, z);
    while (it < max_iter) {
        orc_spmv(n, rp, col, val, p, q);
        double sigma = orc_dot(n, p, q);
        if (!isfinite(sigma)) { status = ORC_NONFINITE; break; }
        if (!(sigma > 0.0)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / sigma;
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        if (alphas) alphas[it] = alpha;
        ++it;
        rnorm = nrm2(n, r);
        if (!isfinite(rnorm)) { status = ORC_NONFINITE; break; }
        if (rnorm <= tol) { status = ORC_OK; break; }
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) z[i] = precond == ORC_PRECOND_JACOBI ? dinv[i] * r[i] : r[i];
        double rho_new = orc_dot(n, r, z);
        double beta = rho_new / rho;
        if (betas) betas[it - 1] = beta;
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = bnorm > 0 ? orc_residual_norm(n, rp, col, val, b, x) / bnorm
                                            : orc_residual_norm(n, rp, col, val, b, x);
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* BiCGStab, right Jacobi preconditioning                                    */
/* ------------------------------------------------------------------------ */
/*
 * x = 0 (or x0); r = b - A x; r_hat = r; rho = alpha = omega = 1; v = p = 0.
 * repeat: rho' = r_hat.r; beta = (rho'/rho)(alpha/omega);
 *         p = r + beta (p - omega v); p_hat = M^{-1} p; v = A p_hat;
 *         alpha = rho' / (r_hat.v); s = r - alpha v;
 *         ||s|| <= tol: x += alpha p_hat, stop;
 *         s_hat = M^{-1} s; t = A s_hat; omega = (t.s)/(t.t);
 *         x += alpha p_hat + omega s_hat; r = s - omega t; ||r|| <= tol: stop;
 *         rho = rho'.
 * Breakdown (rho' == 0, r_hat.v == 0, t.t == 0 or omega == 0): restart once
 * from the current iterate with r_hat = r, rho = alpha = omega = 1,
 * v = p = 0; a second breakdown returns ORC_BREAKDOWN.
 */
int orc_bicgstab(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                 const double *b, double *x, int precond, int use_x0, double rtol, double atol,
                 int64_t max_iter, int64_t *iters_out, double *relres_out)
{
    size_t bytes = sizeof(double) * (size_t)n;
    double *r = malloc(bytes), *rh = malloc(bytes), *p = malloc(bytes), *v = malloc(bytes);
    double *ph = malloc(bytes), *s = malloc(bytes), *sh = malloc(bytes), *t = malloc(bytes);
    double *dinv = malloc(bytes);
    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    int restarts = 0;
    double bnorm = nrm2(n, b);

    if (precond == ORC_PRECOND_JACOBI) {
        if (orc_jacobi_inverse(n, rp, col, val, dinv) != 0) { status = ORC_BAD_INPUT; goto done; }
    } else {
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) dinv[i] = 1.0;
    }
    if (!use_x0) {
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    }
    orc_spmv(n, rp, col, val, x, t);
    PAR_FOR
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    double tol = rtol * bnorm;
    if (atol > tol) tol = atol;
    double rnorm = nrm2(n, r);
    if (!isfinite(rnorm) || !isfinite(bnorm)) { status = ORC_NONFINITE; goto done; }
    if (rnorm <= tol) { status = ORC_OK; goto done; }

restart:
    PAR_FOR
    for (int32_t i = 0; i < n; ++i) { rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    while (it < max_iter) {
        double rho_new = orc_dot(n, rh, r);
        if (!isfinite(rho_new)) { status = ORC_NONFINITE; break; }
        if (rho_new == 0.0) goto breakdown;
        double beta = (rho_new / rho) * (alpha / omega);
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) ph[i] = precond == ORC_PRECOND_JACOBI ? dinv[i] * p[i] : p[i];
        orc_spmv(n, rp, col, val, ph, v);
        double rv = orc_dot(n, rh, v);
        if (!isfinite(rv)) { status = ORC_NONFINITE; break; }
        if (rv == 0.0) goto breakdown;
        alpha = rho_new / rv;
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        ++it;
        double snorm = nrm2(n, s);
        if (!isfinite(snorm)) { status = ORC_NONFINITE; break; }
        if (snorm <= tol) {
            PAR_FOR
            for (int32_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            PAR_FOR
            for (int32_t i = 0; i < n; ++i) r[i] = s[i];
            status = ORC_OK;
            break;
        }
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) sh[i] = precond == ORC_PRECOND_JACOBI ? dinv[i] * s[i] : s[i];
        orc_spmv(n, rp, col, val, sh, t);
        double tt = orc_dot(n, t, t);
        double ts = orc_dot(n, t, s);
        if (!isfinite(tt) || !isfinite(ts)) { status = ORC_NONFINITE; break; }
        if (tt == 0.0) goto breakdown;
        omega = ts / tt;
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * ph[i] + omega * sh[i];
        PAR_FOR
        for (int32_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rnorm = nrm2(n, r);
        if (!isfinite(rnorm)) { status = ORC_NONFINITE; break; }
        if (rnorm <= tol) { status = ORC_OK; break; }
        if (omega == 0.0) goto breakdown;
        rho = rho_new;
        continue;
    breakdown:
        if (restarts++ == 0) goto restart;
        status = ORC_BREAKDOWN;
        break;
    }
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = bnorm > 0 ? orc_residual_norm(n, rp, col, val, b, x) / bnorm
                                            : orc_residual_norm(n, rp, col, val, b, x);
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Transpose and the adjoint gradient                                        */
/* ------------------------------------------------------------------------ */
/* CSR of A^T by counting sort over columns, visiting A's entries in storage
 * order so that each output row is in ascending column order.  src[k'] is the
 * position in A of the entry stored at position k' of A^T; valT may be NULL. */
void orc_transpose(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                   int32_t *rpT, int32_t *colT, double *valT, int32_t *src)
{
    int32_t nnz = rp[n];
    for (int32_t j = 0; j <= n; ++j) rpT[j] = 0;
    for (int32_t k = 0; k < nnz; ++k) rpT[col[k] + 1] += 1;
    for (int32_t j = 0; j < n; ++j) rpT[j + 1] += rpT[j];
    int32_t *next = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t j = 0; j < n; ++j) next[j] = rpT[j];
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            int32_t dst = next[col[k]]++;
            colT[dst] = i;
            src[dst] = k;
            if (valT) valT[dst] = val[k];
        }
    free(next);
}

/* Eq. adjoint_linear: gA[k] = -lambda[i] * x[col[k]] for entry k in row i. */
void orc_adjoint_grad(int32_t n, const int32_t *rp, const int32_t *col, const double *lambda,
                      const double *x, double *gA)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            gA[k] = -lambda[i] * x[col[k]];
}

/* ------------------------------------------------------------------------ */
/* Dense direct solves (tiny n)                                              */
/* ------------------------------------------------------------------------ */
/* Cholesky A = L L^T of a dense row-major SPD matrix; solves A x = b.
 * Returns -1 if a pivot is not positive. */
int orc_dense_cholesky_solve(int32_t n, const double *A, const double *b, double *x)
{
    double *L = calloc((size_t)n * n, sizeof(double));
    double *y = malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    for (int32_t j = 0; j < n && rc == 0; ++j) {
        double d = A[(size_t)j * n + j];
        for (int32_t k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) { rc = -1; break; }
        double ljj = sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int32_t i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int32_t k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / ljj;
        }
    }
    if (rc == 0) {
        for (int32_t i = 0; i < n; ++i) {
            double s = b[i];
            for (int32_t k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int32_t i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int32_t k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
            x[i] = s / L[(size_t)i * n + i];
        }
    }
    free(L); free(y);
    return rc;
}

/* LU with partial pivoting, P A = L U; solves A x = b (trans == 0) or
 * A^T x = b (trans == 1).  Returns -1 on an exactly singular pivot. */
int orc_dense_lu_solve(int32_t n, const double *A, const double *b, double *x, int trans)
{
    double *M = malloc(sizeof(double) * (size_t)n * n);
    int32_t *piv = malloc(sizeof(int32_t) * (size_t)n);
    double *w = malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    memcpy(M, A, sizeof(double) * (size_t)n * n);
    for (int32_t i = 0; i < n; ++i) piv[i] = i;
    for (int32_t k = 0; k < n; ++k) {
        int32_t pr = k;
        double best = fabs(M[(size_t)k * n + k]);
        for (int32_t i = k + 1; i < n; ++i)
            if (fabs(M[(size_t)i * n + k]) > best) { best = fabs(M[(size_t)i * n + k]); pr = i; }
        if (best == 0.0) { rc = -1; break; }
        if (pr != k) {
            for (int32_t j = 0; j < n; ++j) {
                double tmp = M[(size_t)k * n + j];
                M[(size_t)k * n + j] = M[(size_t)pr * n + j];
                M[(size_t)pr * n + j] = tmp;
            }
            int32_t tp = piv[k]; piv[k] = piv[pr]; piv[pr] = tp;
        }
        for (int32_t i = k + 1; i < n; ++i) {
            double l = M[(size_t)i * n + k] / M[(size_t)k * n + k];
            M[(size_t)i * n + k] = l;
            for (int32_t j = k + 1; j < n; ++j) M[(size_t)i * n + j] -= l * M[(size_t)k * n + j];
        }
    }
    if (rc == 0) {
        if (!trans) {
            /* L U x = P b */
            for (int32_t i = 0; i < n; ++i) {
                double s = b[piv[i]];
                for (int32_t k = 0; k < i; ++k) s -= M[(size_t)i * n + k] * w[k];
                w[i] = s;
            }
            for (int32_t i = n - 1; i >= 0; --i) {
                double s = w[i];
                for (int32_t k = i + 1; k < n; ++k) s -= M[(size_t)i * n + k] * x[k];
                x[i] = s / M[(size_t)i * n + i];
            }
        } else {
            /* A^T = U^T L^T P: U^T y = b, L^T w = y, x = P^T w */
            for (int32_t i = 0; i < n; ++i) {
                double s = b[i];
                for (int32_t k = 0; k < i; ++k) s -= M[(size_t)k * n + i] * w[k];
                w[i] = s / M[(size_t)i * n + i];
            }
            for (int32_t i = n - 1; i >= 0; --i) {
                double s = w[i];
                for (int32_t k = i + 1; k < n; ++k) s -= M[(size_t)k * n + i] * w[k];
                w[i] = s;
            }
            for (int32_t i = 0; i < n; ++i) x[piv[i]] = w[i];
        }
    }
    free(M); free(piv); free(w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Factorized sparse approximate inverse                                     */
/* ------------------------------------------------------------------------ */
/* Lower pattern of A (entries with col <= row), as CSR index arrays plus the
 * position of each lower entry in A.  Returns nnz_L. */
int32_t orc_lower_pattern(int32_t n, const int32_t *rp, const int32_t *col,
                          int32_t *rpL, int32_t *colL, int32_t *posA)
{
    int32_t c = 0;
    rpL[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] <= i) {
                if (colL) colL[c] = col[k];
                if (posA) posA[c] = k;
                ++c;
            }
        rpL[i + 1] = c;
    }
    return c;
}

/* Classical FSAI: for row i with lower pattern P_i (ascending, last = i),
 * solve A[P_i, P_i] g = e_last and set G[i, P_i] = g / sqrt(g_last).  Then
 * diag(G A G^T) = 1.  Returns -1 if a local block is not SPD. */
int orc_fsai(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
             const int32_t *rpL, const int32_t *colL, double *gL)
{
    int rc = 0;
    int32_t maxd = 0;
    for (int32_t i = 0; i < n; ++i)
        if (rpL[i + 1] - rpL[i] > maxd) maxd = rpL[i + 1] - rpL[i];
    double *blk = malloc(sizeof(double) * (size_t)maxd * maxd + 1);
    double *e = malloc(sizeof(double) * (size_t)maxd + 1);
    double *g = malloc(sizeof(double) * (size_t)maxd + 1);
    for (int32_t i = 0; i < n && rc == 0; ++i) {
        int32_t d = rpL[i + 1] - rpL[i];
        const int32_t *P = colL + rpL[i];
        if (d == 0 || P[d - 1] != i) { rc = -1; break; }
        for (int32_t a = 0; a < d; ++a)
            for (int32_t b2 = 0; b2 < d; ++b2) {
                double v = 0.0;
                int32_t r = P[a], c = P[b2];
                for (int32_t k = rp[r]; k < rp[r + 1]; ++k)
                    if (col[k] == c) v = val[k];
                blk[(size_t)a * d + b2] = v;
            }
        for (int32_t a = 0; a < d; ++a) e[a] = 0.0;
        e[d - 1] = 1.0;
        if (orc_dense_cholesky_solve(d, blk, e, g) != 0 || !(g[d - 1] > 0.0)) { rc = -1; break; }
        double s = sqrt(g[d - 1]);
        for (int32_t a = 0; a < d; ++a) gL[rpL[i] + a] = g[a] / s;
    }
    free(blk); free(e); free(g);
    return rc;
}

/* z = G^T (G r) with G lower CSR (rpL, colL, gL). */
void orc_fsai_apply(int32_t n, const int32_t *rpL, const int32_t *colL, const double *gL,
                    const double *r, double *z)
{
    double *w = malloc(sizeof(double) * (size_t)n);
    orc_spmv(n, rpL, colL, gL, r, w);
    for (int32_t j = 0; j < n; ++j) z[j] = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rpL[i]; k < rpL[i + 1]; ++k)
            z[colL[k]] += gL[k] * w[i];
    free(w);
}

/* PCG with the factorized preconditioner M^{-1} = G^T G (same recurrence as
 * orc_cg with z = G^T G r). */
int orc_fsai_pcg(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                 const int32_t *rpL, const int32_t *colL, const double *gL,
                 const double *b, double *x, double rtol, double atol, int64_t max_iter,
                 int64_t *iters_out, double *relres_out)
{
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    double bnorm = nrm2(n, b);
    double tol = rtol * bnorm;
    if (atol > tol) tol = atol;
    for (int32_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    double rnorm = bnorm;
    if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
    if (rnorm <= tol) { status = ORC_OK; goto done; }
    orc_fsai_apply(n, rpL, colL, gL, r, z);
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = orc_dot(n, r, z);
    while (it < max_iter) {
        orc_spmv(n, rp, col, val, p, q);
        double sigma = orc_dot(n, p, q);
        if (!isfinite(sigma)) { status = ORC_NONFINITE; break; }
        if (!(sigma > 0.0)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / sigma;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        ++it;
        rnorm = nrm2(n, r);
        if (!isfinite(rnorm)) { status = ORC_NONFINITE; break; }
        if (rnorm <= tol) { status = ORC_OK; break; }
        orc_fsai_apply(n, rpL, colL, gL, r, z);
        double rho_new = orc_dot(n, r, z);
        double beta = rho_new / rho;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = bnorm > 0 ? orc_residual_norm(n, rp, col, val, b, x) / bnorm : 0.0;
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Probe loss of a factorized approximate inverse                            */
/* ------------------------------------------------------------------------ */
/* For each of the P probes z (row-major [P][n]):
 *   w = G^T z, u = A w, v = G u, e = v - z, loss += ||e||^2;
 *   dloss/dG_ij += 2 (e_i u_j + z_i y_j) on G's pattern, y = A^T G^T e.
 * Returns the sum over probes (no normalisation); gG may be NULL. */
double orc_probe_loss(int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                      const int32_t *rpL, const int32_t *colL, const double *gL,
                      int32_t P, const double *Z, double *gG)
{
    size_t bytes = sizeof(double) * (size_t)n;
    double *w = malloc(bytes), *u = malloc(bytes), *v = malloc(bytes), *e = malloc(bytes);
    double *gte = malloc(bytes), *y = malloc(bytes);
    int32_t nnzA = rp[n];
    int32_t *rpT = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *colT = malloc(sizeof(int32_t) * (size_t)(nnzA > 0 ? nnzA : 1));
    double *valT = malloc(sizeof(double) * (size_t)(nnzA > 0 ? nnzA : 1));
    int32_t *srcT = malloc(sizeof(int32_t) * (size_t)(nnzA > 0 ? nnzA : 1));
    orc_transpose(n, rp, col, val, rpT, colT, valT, srcT);
    double loss = 0.0;
    if (gG)
        for (int32_t k = 0; k < rpL[n]; ++k) gG[k] = 0.0;
    for (int32_t pi = 0; pi < P; ++pi) {
        const double *z = Z + (size_t)pi * n;
        /* w = G^T z */
        for (int32_t j = 0; j < n; ++j) w[j] = 0.0;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = rpL[i]; k < rpL[i + 1]; ++k) w[colL[k]] += gL[k] * z[i];
        orc_spmv(n, rp, col, val, w, u);
        orc_spmv(n, rpL, colL, gL, u, v);
        for (int32_t i = 0; i < n; ++i) e[i] = v[i] - z[i];
        loss += orc_dot(n, e, e);
        if (gG) {
            for (int32_t j = 0; j < n; ++j) gte[j] = 0.0;
            for (int32_t i = 0; i < n; ++i)
                for (int32_t k = rpL[i]; k < rpL[i + 1]; ++k) gte[colL[k]] += gL[k] * e[i];
            orc_spmv(n, rpT, colT, valT, gte, y);
            for (int32_t i = 0; i < n; ++i)
                for (int32_t k = rpL[i]; k < rpL[i + 1]; ++k)
                    gG[k] += 2.0 * (e[i] * u[colL[k]] + z[i] * y[colL[k]]);
        }
    }
    free(w); free(u); free(v); free(e); free(gte); free(y);
    free(rpT); free(colT); free(valT); free(srcT);
    return loss;
}
