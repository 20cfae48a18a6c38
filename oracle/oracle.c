/*
 * oracle.c -- plain, slow, FP64 CPU oracle for deflated restarted GMRES(m).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU solver; both sides only take their inputs
 * from the seeded workload generator.
 *
 * What it computes (arXiv 1906.04051):
 *   - CSR sparse matrix-vector product (Sec. 4, CSR storage);
 *   - GMRES(m): Arnoldi with modified Gram-Schmidt (Sec. 3.2, eq. krylov-basis),
 *     plane (Givens) rotations of the Hessenberg matrix and the residual
 *     by-product |gamma_{k+1}| (eqs. arg, hessenberg, res), solution update
 *     x_m = x_0 + V_m y_m (eq. new_sol), restarts from x_m and the relative
 *     residual test ||r||/||r0|| on the true residual (eq. relative);
 *   - deflation with a fixed basis Z: P = I - A Z E^{-1} Z^T, E = Z^T A Z
 *     (the coarse matrix plays the role of T_r = U^T A U, eq. tau_mat), solved
 *     with a dense LU with partial pivoting.  GMRES iterates on P A xh = P b
 *     and returns x = xh + Z E^{-1} Z^T (b - A xh), which is equivalent to
 *     right-preconditioned GMRES (eq. precond1) with a coarse correction.
 *
 * Readings where the paper is silent (stated once here, used below):
 *   - rho0 = ||b - A x0||_2 (undeflated), stop when ||P(b - A xh)|| <= rtol*rho0;
 *   - "iterations" counts inner Arnoldi steps over all restarts;
 *   - lucky breakdown when h_{j+1,j} <= eps * ||w before orthogonalisation||;
 *   - Givens: rho = hypot(a, b), c = a/rho, s = b/rho;
 *   - rtol = 0 runs exactly max_iters inner steps (the paper's fixed-count
 *     protocol, Sec. 4: 50 inner x 100 outer, no termination test).
 * Build with -ffp-contract=off; sums run in index order.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_MAXITER = 1, OR_EINVAL = -1, OR_ESINGULAR = -2, OR_ENONFINITE = -3, OR_ENOMEM = -6 };

/* ---------------------------------------------------------------- basics */

/* y = A x, A in CSR: y_i = sum_k vals[k] x[colind[k]] for k in row i. */
void oracle_spmv(int64_t n, const int32_t *rowptr, const int32_t *colind,
                 const double *vals, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += vals[k] * x[colind[k]];
        y[i] = s;
    }
}

double oracle_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

double oracle_nrm2(int64_t n, const double *a)
{
    return sqrt(oracle_dot(n, a, a));
}

/* In-place LU with partial pivoting of the row-major r x r matrix E
 * (Doolittle; unit lower L below the diagonal, U on and above).
 * piv[k] = row swapped with row k at step k.
 * Returns OR_ESINGULAR when |pivot| <= r * eps * max|E_ij|. */
int oracle_lu_factor(int32_t r, double *E, int32_t *piv)
{
    double emax = 0.0;
    for (int64_t i = 0; i < (int64_t)r * r; ++i)
        if (fabs(E[i]) > emax) emax = fabs(E[i]);
    const double tiny = (double)r * DBL_EPSILON * emax;
    for (int32_t k = 0; k < r; ++k) {
        int32_t p = k;
        for (int32_t i = k + 1; i < r; ++i)
            if (fabs(E[(int64_t)i * r + k]) > fabs(E[(int64_t)p * r + k])) p = i;
        piv[k] = p;
        if (!(fabs(E[(int64_t)p * r + k]) > tiny)) return OR_ESINGULAR;
        if (p != k)
            for (int32_t j = 0; j < r; ++j) {
                double t = E[(int64_t)k * r + j];
                E[(int64_t)k * r + j] = E[(int64_t)p * r + j];
                E[(int64_t)p * r + j] = t;
            }
        for (int32_t i = k + 1; i < r; ++i) {
            double l = E[(int64_t)i * r + k] / E[(int64_t)k * r + k];
            E[(int64_t)i * r + k] = l;
            for (int32_t j = k + 1; j < r; ++j)
                E[(int64_t)i * r + j] -= l * E[(int64_t)k * r + j];
        }
    }
    return OR_OK;
}

/* Solve (P L U) s = t in place: apply the row swaps, then L, then U. */
void oracle_lu_solve(int32_t r, const double *LU, const int32_t *piv, double *x)
{
    for (int32_t k = 0; k < r; ++k)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int32_t i = 0; i < r; ++i)
        for (int32_t j = 0; j < i; ++j)
            x[i] -= LU[(int64_t)i * r + j] * x[j];
    for (int32_t i = r - 1; i >= 0; --i) {
        for (int32_t j = i + 1; j < r; ++j)
            x[i] -= LU[(int64_t)i * r + j] * x[j];
        x[i] /= LU[(int64_t)i * r + i];
    }
}

/* ------------------------------------------------------------- deflation */

typedef struct {
    int64_t n;
    int32_t r;
    const int32_t *zrp, *zci;
    const double *zv;
    double *AZ;       /* n x r, column k at AZ + k*n */
    double *LU;       /* r x r */
    int32_t *piv;
    double *t;        /* r scratch */
} oracle_defl;

/* AZ = A Z column by column, E = Z^T (A Z), LU(E). */
static int defl_setup(oracle_defl *d, int64_t n, const int32_t *rowptr, const int32_t *colind,
                      const double *vals, int32_t r, const int32_t *zrp, const int32_t *zci,
                      const double *zv)
{
    memset(d, 0, sizeof(*d));
    d->n = n; d->r = r; d->zrp = zrp; d->zci = zci; d->zv = zv;
    if (r == 0) return OR_OK;
    d->AZ = (double *)calloc((size_t)n * r, sizeof(double));
    d->LU = (double *)calloc((size_t)r * r, sizeof(double));
    d->piv = (int32_t *)calloc((size_t)r, sizeof(int32_t));
    d->t = (double *)calloc((size_t)r, sizeof(double));
    double *zk = (double *)calloc((size_t)n, sizeof(double));
    if (!d->AZ || !d->LU || !d->piv || !d->t || !zk) { free(zk); return OR_ENOMEM; }
    for (int32_t k = 0; k < r; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            zk[i] = 0.0;
            for (int32_t q = zrp[i]; q < zrp[i + 1]; ++q)
                if (zci[q] == k) zk[i] += zv[q];
        }
        oracle_spmv(n, rowptr, colind, vals, zk, d->AZ + (size_t)k * n);
    }
    free(zk);
    /* E[a][k] = sum_i Z[i][a] AZ[i][k] */
    for (int64_t i = 0; i < n; ++i)
        for (int32_t q = zrp[i]; q < zrp[i + 1]; ++q)
            for (int32_t k = 0; k < r; ++k)
                d->LU[(int64_t)zci[q] * r + k] += zv[q] * d->AZ[(size_t)k * n + i];
    return oracle_lu_factor(r, d->LU, d->piv);
}

static void defl_free(oracle_defl *d)
{
    free(d->AZ); free(d->LU); free(d->piv); free(d->t);
}

/* s = E^{-1} Z^T y  (into d->t) */
static void defl_coarse(const oracle_defl *d, const double *y)
{
    for (int32_t k = 0; k < d->r; ++k) d->t[k] = 0.0;
    for (int64_t i = 0; i < d->n; ++i)
        for (int32_t q = d->zrp[i]; q < d->zrp[i + 1]; ++q)
            d->t[d->zci[q]] += d->zv[q] * y[i];
    oracle_lu_solve(d->r, d->LU, d->piv, d->t);
}

/* w = P y = y - A Z E^{-1} Z^T y */
static void defl_apply_P(const oracle_defl *d, const double *y, double *w)
{
    if (d->r == 0) { memcpy(w, y, sizeof(double) * (size_t)d->n); return; }
    defl_coarse(d, y);
    for (int64_t i = 0; i < d->n; ++i) {
        double s = y[i];
        for (int32_t k = 0; k < d->r; ++k)
            s -= d->AZ[(size_t)k * d->n + i] * d->t[k];
        w[i] = s;
    }
}

/* x += Z E^{-1} Z^T r  (the coarse correction Q r) */
static void defl_correct(const oracle_defl *d, const double *r, double *x)
{
    if (d->r == 0) return;
    defl_coarse(d, r);
    for (int64_t i = 0; i < d->n; ++i)
        for (int32_t q = d->zrp[i]; q < d->zrp[i + 1]; ++q)
            x[i] += d->zv[q] * d->t[d->zci[q]];
}

/* The same operator for the block oracle (bgmres.c), as an opaque handle:
 * create (NULL and *status != OR_OK on failure), w = P y, x += Z E^{-1} Z^T r,
 * destroy. */
void *oracle_defl_create(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                         int32_t r, const int32_t *zrp, const int32_t *zci, const double *zv,
                         int *status)
{
    oracle_defl *d = (oracle_defl *)calloc(1, sizeof(oracle_defl));
    if (!d) {
        *status = OR_ENOMEM;
        return NULL;
    }
    *status = defl_setup(d, n, rowptr, colind, vals, r, zrp, zci, zv);
    if (*status != OR_OK) {
        defl_free(d);
        free(d);
        return NULL;
    }
    return d;
}

void oracle_defl_apply(void *d, const double *y, double *w) { defl_apply_P((const oracle_defl *)d, y, w); }

void oracle_defl_correct(void *d, const double *r, double *x) { defl_correct((const oracle_defl *)d, r, x); }

void oracle_defl_destroy(void *d)
{
    if (!d) return;
    defl_free((oracle_defl *)d);
    free(d);
}

/* Exposed for tests: w = P y for one vector (sets up and frees the coarse
 * operator on each call). */
int oracle_apply_projector(int64_t n, const int32_t *rowptr, const int32_t *colind,
                           const double *vals, int32_t r, const int32_t *zrp,
                           const int32_t *zci, const double *zv, const double *y, double *w)
{
    oracle_defl d;
    int st = defl_setup(&d, n, rowptr, colind, vals, r, zrp, zci, zv);
    if (st == OR_OK) defl_apply_P(&d, y, w);
    defl_free(&d);
    return st;
}

/* ------------------------------------------------------------------ GMRES */

static int all_finite(int64_t n, const double *v)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/*
 * Deflated GMRES(m).
 *   x0 may be NULL (zero initial guess).  x receives the coarse-corrected
 *   solution.  info_i = {iters, cycles, status}; info_d = {rho0,
 *   rel_res_deflated (= ||P(b - A xh)|| / rho0 at exit), rel_res_true
 *   (= ||b - A x|| / rho0 recomputed)}.
 *   hist (optional, length max_iters): |gamma_{k+1}| after every inner step.
 *   V0 (optional, n x (m+1), column j at V0 + j*n) and H0 (optional,
 *   (m+1) x m row-major, before rotations): the first cycle's basis and
 *   Hessenberg matrix, for invariant checks.
 */
int oracle_gmres(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                 const double *b, const double *x0,
                 int32_t r, const int32_t *zrp, const int32_t *zci, const double *zv,
                 int32_t m, int64_t max_iters, double rtol, double r0_norm_override,
                 double *x, int64_t *info_i, double *info_d,
                 double *hist, double *V0, double *H0)
{
    info_i[0] = 0; info_i[1] = 0; info_i[2] = OR_EINVAL;
    info_d[0] = info_d[1] = info_d[2] = 0.0;
    if (n <= 0 || m <= 0 || max_iters < 0 || !(rtol >= 0.0) || r < 0) return OR_EINVAL;
    if (!all_finite(rowptr[n], vals) || !all_finite(n, b) || (x0 && !all_finite(n, x0))) {
        info_i[2] = OR_ENONFINITE;
        return OR_ENONFINITE;
    }
    oracle_defl d;
    int st = defl_setup(&d, n, rowptr, colind, vals, r, zrp, zci, zv);
    if (st != OR_OK) { defl_free(&d); info_i[2] = st; return st; }

    double *V = (double *)calloc((size_t)n * (m + 1), sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));   /* H[i*m + j] */
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *yv = (double *)calloc((size_t)m, sizeof(double));
    double *rv = (double *)calloc((size_t)n, sizeof(double));
    double *tmp = (double *)calloc((size_t)n, sizeof(double));
    if (!V || !H || !cs || !sn || !g || !yv || !rv || !tmp) {
        st = OR_ENOMEM;
        goto done;
    }

    /* x_hat = x0 ; r0 = b - A x0 ; rho0 = ||r0|| (eq. relative) */
    for (int64_t i = 0; i < n; ++i) x[i] = x0 ? x0[i] : 0.0;
    oracle_spmv(n, rowptr, colind, vals, x, tmp);
    for (int64_t i = 0; i < n; ++i) rv[i] = b[i] - tmp[i];
    double rho0 = oracle_nrm2(n, rv);
    if (r0_norm_override > 0.0) rho0 = r0_norm_override;
    info_d[0] = rho0;
    if (rho0 == 0.0) {
        st = OR_OK;
        info_d[1] = info_d[2] = 0.0;
        goto done;
    }
    const double target = rtol * rho0;
    int64_t its = 0;
    int64_t cycles = 0;
    int first_cycle = 1;
    double beta;

    for (;;) {
        /* Restart: true residual of the current iterate, deflated. */
        oracle_spmv(n, rowptr, colind, vals, x, tmp);
        for (int64_t i = 0; i < n; ++i) rv[i] = b[i] - tmp[i];
        defl_apply_P(&d, rv, V);                      /* p = P r into V[:,0] */
        beta = oracle_nrm2(n, V);
        if (beta <= target) { st = OR_OK; break; }
        if (its >= max_iters) { st = OR_MAXITER; break; }
        ++cycles;
        for (int64_t i = 0; i < n; ++i) V[i] /= beta;   /* v1 = p / beta */
        for (int32_t i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;                                     /* g = beta e1 (eq. arg) */
        int32_t k = 0;
        for (int32_t j = 0; j < m && its < max_iters; ++j) {
            double *vj = V + (size_t)j * n;
            double *w = V + (size_t)(j + 1) * n;
            /* w = P A v_j */
            oracle_spmv(n, rowptr, colind, vals, vj, tmp);
            defl_apply_P(&d, tmp, w);
            ++its;
            double wpre = oracle_nrm2(n, w);
            /* Modified Gram-Schmidt (Sec. 3.2) */
            for (int32_t i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * n;
                double hij = oracle_dot(n, vi, w);
                H[(int64_t)i * m + j] = hij;
                for (int64_t q = 0; q < n; ++q) w[q] -= hij * vi[q];
            }
            double hn = oracle_nrm2(n, w);
            H[(int64_t)(j + 1) * m + j] = hn;
            int breakdown = !(hn > DBL_EPSILON * wpre);
            if (!breakdown)
                for (int64_t q = 0; q < n; ++q) w[q] /= hn;
            if (first_cycle && H0)
                for (int32_t i = 0; i <= j + 1; ++i) H0[(int64_t)i * m + j] = H[(int64_t)i * m + j];
            /* Previous rotations applied to column j, then the new one. */
            for (int32_t i = 0; i < j; ++i) {
                double a = H[(int64_t)i * m + j], c = H[(int64_t)(i + 1) * m + j];
                H[(int64_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(int64_t)j * m + j], c = H[(int64_t)(j + 1) * m + j];
            double rho = hypot(a, c);
            if (c == 0.0) { cs[j] = 1.0; sn[j] = 0.0; rho = a; }
            else { cs[j] = a / rho; sn[j] = c / rho; }
            H[(int64_t)j * m + j] = rho;
            H[(int64_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            if (hist) hist[its - 1] = fabs(g[j + 1]);
            k = j + 1;
            if (fabs(g[j + 1]) <= target || breakdown) break;
        }
        if (first_cycle && V0)
            memcpy(V0, V, sizeof(double) * (size_t)n * (k + 1));
        first_cycle = 0;
        /* Back substitution R_k y = g_{1:k}; x_hat += V_k y (eq. new_sol) */
        for (int32_t i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int32_t q = i + 1; q < k; ++q) s -= H[(int64_t)i * m + q] * yv[q];
            yv[i] = s / H[(int64_t)i * m + i];
        }
        for (int32_t i = 0; i < k; ++i) {
            const double *vi = V + (size_t)i * n;
            for (int64_t q = 0; q < n; ++q) x[q] += yv[i] * vi[q];
        }
    }
    info_i[0] = its;
    info_i[1] = cycles;
    info_d[1] = beta / rho0;

    /* x = x_hat + Z E^{-1} Z^T (b - A x_hat); rv already holds b - A x_hat. */
    defl_correct(&d, rv, x);
    oracle_spmv(n, rowptr, colind, vals, x, tmp);
    for (int64_t i = 0; i < n; ++i) tmp[i] = b[i] - tmp[i];
    info_d[2] = oracle_nrm2(n, tmp) / rho0;

done:
    info_i[2] = st;
    free(V); free(H); free(cs); free(sn); free(g); free(yv); free(rv); free(tmp);
    defl_free(&d);
    return st;
}

/* ---------------------------------------------------------------- adjoint */

/* CSR transpose by counting: row j of A^T holds the entries of column j of A,
 * in increasing original row order. */
void oracle_csr_transpose(int64_t n, const int32_t *rowptr, const int32_t *colind,
                          const double *vals, int32_t *trowptr, int32_t *tcolind, double *tvals)
{
    int32_t nnz = rowptr[n];
    for (int64_t j = 0; j <= n; ++j) trowptr[j] = 0;
    for (int32_t k = 0; k < nnz; ++k) trowptr[colind[k] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) trowptr[j + 1] += trowptr[j];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) fill[j] = trowptr[j];
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int32_t pos = fill[colind[k]]++;
            tcolind[pos] = (int32_t)i;
            tvals[pos] = vals[k];
        }
    free(fill);
}

/* dL/dA_ij = -lambda_i x_j on A's pattern (derivative of x = A^{-1} b). */
void oracle_grad_vals(int64_t n, const int32_t *rowptr, const int32_t *colind,
                      const double *lambda, const double *x, double *grad)
{
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            grad[k] = -lambda[i] * x[colind[k]];
}
