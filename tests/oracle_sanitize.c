/*
 * Driver for the address/undefined-behaviour sanitizer build of the CPU
 * oracle (test infrastructure).  Runs every exported oracle routine on
 * small matrices -- the 2D Poisson operator, a nonsymmetric upwind variant,
 * a pattern with an empty row and explicit zeros, n = 1 and n = 0 -- with
 * one and with several threads, and checks a few results that hold
 * exactly.  Exit status 0 means no sanitizer report and every check held.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_set_threads(int threads);
void orc_spmv(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const double *x, double *y);
double orc_dot(int64_t n, const double *a, const double *b);
int orc_jacobi_inverse(int32_t n, const int32_t *rp, const int32_t *col, const double *val, double *dinv);
double orc_residual_norm(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const double *b,
                         const double *x);
int orc_cg(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const double *b, double *x,
           int precond, int use_x0, double rtol, double atol, int64_t max_iter, int64_t *iters_out,
           double *relres_out, double *alphas, double *betas);
int orc_bicgstab(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const double *b, double *x,
                 int precond, int use_x0, double rtol, double atol, int64_t max_iter, int64_t *iters_out,
                 double *relres_out);
void orc_transpose(int32_t n, const int32_t *rp, const int32_t *col, const double *val, int32_t *rpT,
                   int32_t *colT, double *valT, int32_t *src);
void orc_adjoint_grad(int32_t n, const int32_t *rp, const int32_t *col, const double *lambda, const double *x,
                      double *gA);
int orc_dense_cholesky_solve(int32_t n, const double *A, const double *b, double *x);
int orc_dense_lu_solve(int32_t n, const double *A, const double *b, double *x, int trans);
int32_t orc_lower_pattern(int32_t n, const int32_t *rp, const int32_t *col, int32_t *rpL, int32_t *colL,
                          int32_t *posA);
int orc_fsai(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const int32_t *rpL,
             const int32_t *colL, double *gL);
void orc_fsai_apply(int32_t n, const int32_t *rpL, const int32_t *colL, const double *gL, const double *r,
                    double *z);
int orc_fsai_pcg(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const int32_t *rpL,
                 const int32_t *colL, const double *gL, const double *b, double *x, double rtol, double atol,
                 int64_t max_iter, int64_t *iters_out, double *relres_out);
double orc_probe_loss(int32_t n, const int32_t *rp, const int32_t *col, const double *val, const int32_t *rpL,
                      const int32_t *colL, const double *gL, int32_t P, const double *Z, double *gG);

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

typedef struct {
    int32_t n;
    int32_t *rp, *col;
    double *val;
} Csr;

/* m x m 5-point operator (diag 4 + shift, off -1); `up` > 0 adds upwind
 * convection (nonsymmetric). */
static Csr poisson(int32_t m, double shift, double up) {
    Csr a;
    a.n = m * m;
    a.rp = malloc(sizeof(int32_t) * (size_t)(a.n + 1));
    a.col = malloc(sizeof(int32_t) * (size_t)(5 * a.n));
    a.val = malloc(sizeof(double) * (size_t)(5 * a.n));
    int32_t k = 0;
    a.rp[0] = 0;
    for (int32_t y = 0; y < m; ++y)
        for (int32_t x = 0; x < m; ++x) {
            const int32_t i = y * m + x;
            if (y > 0) { a.col[k] = i - m; a.val[k++] = -1.0 - up; }
            if (x > 0) { a.col[k] = i - 1; a.val[k++] = -1.0 - up; }
            a.col[k] = i; a.val[k++] = 4.0 + shift + 2.0 * up;
            if (x < m - 1) { a.col[k] = i + 1; a.val[k++] = -1.0; }
            if (y < m - 1) { a.col[k] = i + m; a.val[k++] = -1.0; }
            a.rp[i + 1] = k;
        }
    return a;
}

static void free_csr(Csr *a) {
    free(a->rp);
    free(a->col);
    free(a->val);
}

static void run_all(const Csr *a, int sym) {
    const int32_t n = a->n, nnz = a->rp[n];
    const size_t nb = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *b = malloc(nb), *x = malloc(nb), *y = malloc(nb), *d = malloc(nb), *lam = malloc(nb);
    double *gA = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    for (int32_t i = 0; i < n; ++i) b[i] = sin(1.0 + i);
    int64_t it = 0;
    double rr = 0.0;
    double *al = malloc(sizeof(double) * 4096), *be = malloc(sizeof(double) * 4096);
    if (sym) {
        CHECK(orc_cg(n, a->rp, a->col, a->val, b, x, 0, 0, 1e-10, 0.0, 4096, &it, &rr, al, be) == 0);
        CHECK(orc_cg(n, a->rp, a->col, a->val, b, x, 1, 1, 1e-12, 0.0, 4096, &it, &rr, NULL, NULL) == 0);
    }
    CHECK(orc_bicgstab(n, a->rp, a->col, a->val, b, x, 1, 0, 1e-10, 0.0, 4096, &it, &rr) == 0);
    CHECK(orc_residual_norm(n, a->rp, a->col, a->val, b, x) <= 1e-9 * sqrt(orc_dot(n, b, b)) + 1e-300);
    orc_spmv(n, a->rp, a->col, a->val, x, y);
    CHECK(orc_jacobi_inverse(n, a->rp, a->col, a->val, d) == 0);
    int32_t *rpT = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *colT = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *src = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *valT = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    orc_transpose(n, a->rp, a->col, a->val, rpT, colT, valT, src);
    for (int32_t k = 0; k < nnz; ++k) CHECK(valT[k] == a->val[src[k]]);
    for (int32_t i = 0; i < n; ++i) lam[i] = cos(0.5 * i);
    orc_adjoint_grad(n, a->rp, a->col, lam, x, gA);
    if (sym && n > 0) {
        int32_t *rpL = malloc(sizeof(int32_t) * (size_t)(n + 1));
        const int32_t nL = orc_lower_pattern(n, a->rp, a->col, rpL, NULL, NULL);
        int32_t *colL = malloc(sizeof(int32_t) * (size_t)nL), *pos = malloc(sizeof(int32_t) * (size_t)nL);
        orc_lower_pattern(n, a->rp, a->col, rpL, colL, pos);
        double *g = malloc(sizeof(double) * (size_t)nL), *gG = malloc(sizeof(double) * (size_t)nL);
        CHECK(orc_fsai(n, a->rp, a->col, a->val, rpL, colL, g) == 0);
        orc_fsai_apply(n, rpL, colL, g, b, y);
        CHECK(orc_fsai_pcg(n, a->rp, a->col, a->val, rpL, colL, g, b, x, 1e-10, 0.0, 4096, &it, &rr) == 0);
        double *Z = malloc(nb * 3);
        for (int32_t i = 0; i < 3 * n; ++i) Z[i] = (i * 7919 % 3 == 0) ? -1.0 : 1.0;
        CHECK(orc_probe_loss(n, a->rp, a->col, a->val, rpL, colL, g, 3, Z, gG) >= 0.0);
        free(rpL); free(colL); free(pos); free(g); free(gG); free(Z);
    }
    if (n > 0 && n <= 64) {
        double *A = calloc((size_t)n * n, sizeof(double));
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = a->rp[i]; k < a->rp[i + 1]; ++k) A[(size_t)i * n + a->col[k]] = a->val[k];
        if (sym) CHECK(orc_dense_cholesky_solve(n, A, b, y) == 0);
        CHECK(orc_dense_lu_solve(n, A, b, y, 0) == 0);
        CHECK(orc_dense_lu_solve(n, A, b, y, 1) == 0);
        free(A);
    }
    free(b); free(x); free(y); free(d); free(lam); free(gA); free(al); free(be);
    free(rpT); free(colT); free(src); free(valT);
}

int main(void) {
    const int threads[2] = {1, 4};
    for (int t = 0; t < 2; ++t) {
        orc_set_threads(threads[t]);
        Csr a = poisson(7, 0.0, 0.0);
        run_all(&a, 1);
        free_csr(&a);
        a = poisson(9, 0.5, 0.7);
        run_all(&a, 0);
        free_csr(&a);
        a = poisson(1, 0.0, 0.0);  /* n = 1 */
        run_all(&a, 1);
        free_csr(&a);
        /* explicit zeros and an empty row under SpMV and transpose only */
        int32_t rp[4] = {0, 2, 2, 4}, col[4] = {0, 2, 0, 2};
        double val[4] = {2.0, 0.0, 0.0, 3.0}, xv[3] = {1.0, 2.0, 3.0}, yv[3];
        orc_spmv(3, rp, col, val, xv, yv);
        CHECK(yv[0] == 2.0 && yv[1] == 0.0 && yv[2] == 9.0);
        int32_t rpT[4], colT[4], src[4];
        double valT[4];
        orc_transpose(3, rp, col, val, rpT, colT, valT, src);
        CHECK(rpT[3] == 4);
        /* n = 0 */
        int32_t rp0[1] = {0};
        double e[1];
        orc_spmv(0, rp0, col, val, e, e);
        orc_transpose(0, rp0, col, val, rpT, colT, valT, src);
    }
    if (failures) return 1;
    printf("oracle sanitizer run: all checks held\n");
    return 0;
}
