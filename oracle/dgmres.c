/*
 * dgmres.c -- plain FP64 CPU oracle for GMRES(m) right-preconditioned by the
 * paper's adaptive spectral deflation (arXiv 1906.04051, Sec. 3.3).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library.
 *
 * What it computes:
 *   - right preconditioning A M^{-1} z = b, x = M^{-1} z (eq. precond1) with
 *     M^{-1} = I + U (|mu| T^{-1} - I) U^T (eq. precond2), T = U^T A U
 *     (eq. tau_mat), U orthonormal (N x r);
 *   - GMRES(m) on A M^{-1} (MGS Arnoldi, Givens, |gamma_{k+1}| as in oracle.c);
 *     a cycle updates the iterate in x-space, x += M^{-1} V_k y_k (eq. new_sol
 *     for the right-preconditioned system), so M may change between cycles;
 *   - at every restart (Sec. 3.3): |mu| and one eigenvector z of H_k for its
 *     smallest eigenvalue (l = 1), u = V_k z (eq. precond3) orthonormalised
 *     against U and appended, A u appended to AU, T extended; when r exceeds
 *     r_max the direction of U that belongs to the largest eigenvalue of T
 *     is removed.
 *
 * Readings where the paper is silent (the GPU path uses the same ones):
 *   - |mu|: KPOW = 30 power iterations on H_k from the normalised ones vector,
 *     |mu| = ||H_k z||;
 *   - smallest eigenvector: KINV = 20 inverse iterations on H_k (LU with
 *     partial pivoting) from the normalised ones vector; no append when H_k is
 *     singular (|pivot| <= k eps max|H_k|);
 *   - u is orthonormalised against U by classical Gram-Schmidt applied twice
 *     and appended only when ||u|| > 1e-8 after it (||V_k z|| = 1 before);
 *   - removal: eigenvector w of T for its largest eigenvalue by KPOW power
 *     iterations from the normalised ones vector; the Householder reflection
 *     Q with Q w = alpha e_1 (alpha = -sign(w_1) ||w||) rotates U, AU and T
 *     (U Q, AU Q, Q T Q) and the first column/row is dropped;
 *   - C = |mu| T^{-1} - I from an LU with partial pivoting of T; when T is
 *     singular C = 0 (no preconditioning) until the next restart;
 *   - the starting vector, iteration counts and thresholds above are fixed
 *     constants, so the computation is deterministic.
 * Build with -ffp-contract=off; sums run in index order.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_MAXITER 1
#define OR_EINVAL -1
#define OR_ENONFINITE -3
#define OR_ENOMEM -6

#define KPOW 30
#define KINV 20
#define APPEND_TOL 1e-8

void oracle_spmv(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                 const double *x, double *y);
double oracle_dot(int64_t n, const double *a, const double *b);
double oracle_nrm2(int64_t n, const double *a);
int oracle_lu_factor(int32_t r, double *E, int32_t *piv);
void oracle_lu_solve(int32_t r, const double *LU, const int32_t *piv, double *x);

/* z <- normalised dominant direction of the k x k row-major matrix M after
 * KPOW power iterations from ones/sqrt(k); returns ||M z|| (0 when an iterate
 * vanishes). */
static double power_iteration(int32_t k, const double *M, double *z, double *tmp)
{
    for (int32_t i = 0; i < k; ++i) z[i] = 1.0 / sqrt((double)k);
    for (int it = 0; it < KPOW; ++it) {
        for (int32_t i = 0; i < k; ++i) {
            double s = 0.0;
            for (int32_t q = 0; q < k; ++q) s += M[(int64_t)i * k + q] * z[q];
            tmp[i] = s;
        }
        double nz = 0.0;
        for (int32_t i = 0; i < k; ++i) nz += tmp[i] * tmp[i];
        nz = sqrt(nz);
        if (nz == 0.0) return 0.0;
        for (int32_t i = 0; i < k; ++i) z[i] = tmp[i] / nz;
    }
    double s2 = 0.0;
    for (int32_t i = 0; i < k; ++i) {
        double s = 0.0;
        for (int32_t q = 0; q < k; ++q) s += M[(int64_t)i * k + q] * z[q];
        s2 += s * s;
    }
    return sqrt(s2);
}

/* Exposed for tests: dominant estimate of a k x k row-major matrix. */
double oracle_power_iteration(int32_t k, const double *M, double *z)
{
    double *tmp = (double *)calloc((size_t)k, sizeof(double));
    double mu = tmp ? power_iteration(k, M, z, tmp) : 0.0;
    free(tmp);
    return mu;
}

/* z <- KINV inverse iterations on the k x k row-major matrix M from
 * ones/sqrt(k).  Returns OR_OK, or OR_EINVAL when M is singular. */
int oracle_inverse_iteration(int32_t k, const double *M, double *z)
{
    double *LU = (double *)malloc(sizeof(double) * (size_t)k * k);
    int32_t *piv = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    if (!LU || !piv) { free(LU); free(piv); return OR_ENOMEM; }
    memcpy(LU, M, sizeof(double) * (size_t)k * k);
    int st = oracle_lu_factor(k, LU, piv);
    if (st == OR_OK) {
        for (int32_t i = 0; i < k; ++i) z[i] = 1.0 / sqrt((double)k);
        for (int it = 0; it < KINV; ++it) {
            oracle_lu_solve(k, LU, piv, z);
            double nz = 0.0;
            for (int32_t i = 0; i < k; ++i) nz += z[i] * z[i];
            nz = sqrt(nz);
            for (int32_t i = 0; i < k; ++i) z[i] /= nz;
        }
    } else {
        st = OR_EINVAL;
    }
    free(LU); free(piv);
    return st;
}

typedef struct {
    int64_t n;
    int32_t rmax, r;
    double mu;
    double *U, *AU;   /* n x (rmax+1), column q at + q*n */
    double *T;        /* (rmax+1) x (rmax+1), row-major, leading r x r used */
    double *C;        /* r x r row-major: |mu| T^{-1} - I (zero when T singular) */
    double *t, *s;    /* r-vectors */
} adapt_state;

/* out = M^{-1} v = v + U C U^T v (eq. precond2); out may alias v. */
static void apply_minv(const adapt_state *a, const double *v, double *out)
{
    const int64_t n = a->n;
    const int32_t r = a->r;
    for (int32_t q = 0; q < r; ++q) a->t[q] = oracle_dot(n, a->U + (size_t)q * n, v);
    for (int32_t i = 0; i < r; ++i) {
        double s = 0.0;
        for (int32_t q = 0; q < r; ++q) s += a->C[(int64_t)i * r + q] * a->t[q];
        a->s[i] = s;
    }
    if (out != v) memcpy(out, v, sizeof(double) * (size_t)n);
    for (int32_t q = 0; q < r; ++q) {
        const double *uq = a->U + (size_t)q * n;
        for (int64_t i = 0; i < n; ++i) out[i] += a->s[q] * uq[i];
    }
}

/* C = |mu| T^{-1} - I, column by column through an LU of T. */
static void form_c(adapt_state *a)
{
    const int32_t r = a->r;
    if (r == 0) return;
    double *LU = (double *)malloc(sizeof(double) * (size_t)r * r);
    int32_t *piv = (int32_t *)malloc(sizeof(int32_t) * (size_t)r);
    double *e = (double *)malloc(sizeof(double) * (size_t)r);
    for (int32_t i = 0; i < r; ++i)
        for (int32_t q = 0; q < r; ++q) LU[(int64_t)i * r + q] = a->T[(int64_t)i * (a->rmax + 1) + q];
    if (oracle_lu_factor(r, LU, piv) != OR_OK) {
        memset(a->C, 0, sizeof(double) * (size_t)r * r);
    } else {
        for (int32_t q = 0; q < r; ++q) {
            for (int32_t i = 0; i < r; ++i) e[i] = (i == q) ? 1.0 : 0.0;
            oracle_lu_solve(r, LU, piv, e);
            for (int32_t i = 0; i < r; ++i)
                a->C[(int64_t)i * r + q] = a->mu * e[i] - (i == q ? 1.0 : 0.0);
        }
    }
    free(LU); free(piv); free(e);
}

/* Exposed for tests: out = M^{-1} v for a given orthonormal U (n x r, column
 * q at U + q*n), T (r x r row-major) and |mu| (eq. precond2). */
int oracle_apply_minv(int64_t n, int32_t r, const double *U, const double *T, double mu,
                      const double *v, double *out)
{
    adapt_state a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.rmax = r;
    a.r = r;
    a.mu = mu;
    a.U = (double *)U;
    a.T = (double *)calloc((size_t)(r + 1) * (r + 1), sizeof(double));
    a.C = (double *)calloc((size_t)(r + 1) * (r + 1), sizeof(double));
    a.t = (double *)calloc((size_t)r + 1, sizeof(double));
    a.s = (double *)calloc((size_t)r + 1, sizeof(double));
    if (!a.T || !a.C || !a.t || !a.s) {
        free(a.T); free(a.C); free(a.t); free(a.s);
        return OR_ENOMEM;
    }
    for (int32_t i = 0; i < r; ++i)
        for (int32_t q = 0; q < r; ++q) a.T[(int64_t)i * (r + 1) + q] = T[(int64_t)i * r + q];
    form_c(&a);
    apply_minv(&a, v, out);
    free(a.T); free(a.C); free(a.t); free(a.s);
    return OR_OK;
}

/* One restart's update of the deflation space from the cycle's basis V
 * (k+1 columns) and unrotated Hessenberg H ((m+1) x m row-major). */
static void adapt(adapt_state *a, int64_t n, const int32_t *rowptr, const int32_t *colind,
                  const double *vals, const double *V, const double *H, int32_t m, int32_t k)
{
    const int32_t ld = a->rmax + 1;
    double *Hk = (double *)malloc(sizeof(double) * (size_t)k * k);
    double *z = (double *)malloc(sizeof(double) * (size_t)(k > ld ? k : ld));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(k > ld ? k : ld));
    for (int32_t i = 0; i < k; ++i)
        for (int32_t q = 0; q < k; ++q) Hk[(int64_t)i * k + q] = H[(int64_t)i * m + q];
    a->mu = power_iteration(k, Hk, z, tmp);
    int append = oracle_inverse_iteration(k, Hk, z) == OR_OK;
    if (append) {
        double *u = a->U + (size_t)a->r * n;
        memset(u, 0, sizeof(double) * (size_t)n);
        for (int32_t i = 0; i < k; ++i) {
            const double *vi = V + (size_t)i * n;
            for (int64_t q = 0; q < n; ++q) u[q] += z[i] * vi[q];
        }
        for (int pass = 0; pass < 2; ++pass) {
            for (int32_t q = 0; q < a->r; ++q) tmp[q] = oracle_dot(n, a->U + (size_t)q * n, u);
            for (int32_t q = 0; q < a->r; ++q) {
                const double *uq = a->U + (size_t)q * n;
                for (int64_t i = 0; i < n; ++i) u[i] -= tmp[q] * uq[i];
            }
        }
        const double nu = oracle_nrm2(n, u);
        append = nu > APPEND_TOL;
        if (append) {
            for (int64_t i = 0; i < n; ++i) u[i] /= nu;
            double *au = a->AU + (size_t)a->r * n;
            oracle_spmv(n, rowptr, colind, vals, u, au);
            const int32_t r = a->r;
            for (int32_t q = 0; q <= r; ++q)
                a->T[(int64_t)q * ld + r] = oracle_dot(n, a->U + (size_t)q * n, au);
            for (int32_t q = 0; q < r; ++q)
                a->T[(int64_t)r * ld + q] = oracle_dot(n, u, a->AU + (size_t)q * n);
            a->r = r + 1;
        }
    }
    if (a->r > a->rmax) {
        /* Remove the direction of the largest eigenvalue of T. */
        const int32_t r = a->r;
        double *Tr = (double *)malloc(sizeof(double) * (size_t)r * r);
        double *h = (double *)malloc(sizeof(double) * (size_t)r);
        for (int32_t i = 0; i < r; ++i)
            for (int32_t q = 0; q < r; ++q) Tr[(int64_t)i * r + q] = a->T[(int64_t)i * ld + q];
        power_iteration(r, Tr, z, tmp);
        double nw = 0.0;
        for (int32_t i = 0; i < r; ++i) nw += z[i] * z[i];
        nw = sqrt(nw);
        const double alpha = (z[0] >= 0.0) ? -nw : nw;
        for (int32_t i = 0; i < r; ++i) h[i] = z[i];
        h[0] -= alpha;
        double nh = 0.0;
        for (int32_t i = 0; i < r; ++i) nh += h[i] * h[i];
        nh = sqrt(nh);
        for (int32_t i = 0; i < r; ++i) h[i] /= nh;
        /* U <- U Q, AU <- AU Q (Q = I - 2 h h^T), row by row. */
        double *mats[2] = {a->U, a->AU};
        for (int mi = 0; mi < 2; ++mi) {
            double *Mx = mats[mi];
            for (int64_t i = 0; i < n; ++i) {
                double p = 0.0;
                for (int32_t q = 0; q < r; ++q) p += Mx[(size_t)q * n + i] * h[q];
                for (int32_t q = 0; q < r; ++q) Mx[(size_t)q * n + i] -= 2.0 * p * h[q];
            }
        }
        /* T <- Q T Q */
        for (int32_t i = 0; i < r; ++i) {          /* T Q: rows */
            double p = 0.0;
            for (int32_t q = 0; q < r; ++q) p += Tr[(int64_t)i * r + q] * h[q];
            for (int32_t q = 0; q < r; ++q) Tr[(int64_t)i * r + q] -= 2.0 * p * h[q];
        }
        for (int32_t q = 0; q < r; ++q) {          /* Q (T Q): columns */
            double p = 0.0;
            for (int32_t i = 0; i < r; ++i) p += h[i] * Tr[(int64_t)i * r + q];
            for (int32_t i = 0; i < r; ++i) Tr[(int64_t)i * r + q] -= 2.0 * h[i] * p;
        }
        /* Drop column / row 0. */
        memmove(a->U, a->U + n, sizeof(double) * (size_t)n * (r - 1));
        memmove(a->AU, a->AU + n, sizeof(double) * (size_t)n * (r - 1));
        for (int32_t i = 1; i < r; ++i)
            for (int32_t q = 1; q < r; ++q) a->T[(int64_t)(i - 1) * ld + (q - 1)] = Tr[(int64_t)i * r + q];
        a->r = r - 1;
        free(Tr); free(h);
    }
    form_c(a);
    free(Hk); free(z); free(tmp);
}

static int finite_all(int64_t n, const double *v)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/*
 * Adaptive-deflation GMRES(m).  rmax = 0 gives plain GMRES(m).
 *   info_i = {iters, cycles, status, r at exit}; info_d = {rho0, rel_res
 *   (||b - A x|| / rho0 at the last restart), rel_res_true (recomputed), |mu|}.
 *   hist (optional, length max_iters): |gamma_{k+1}| after every inner step.
 *   Uout (optional, n x rmax) and Tout (optional, rmax x rmax row-major): the
 *   deflation basis and T at exit (leading r columns / r x r).
 */
int oracle_dgmres(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                  const double *b, const double *x0, int32_t m, int64_t max_iters, double rtol,
                  int32_t rmax, double *x, int64_t *info_i, double *info_d, double *hist,
                  double *Uout, double *Tout)
{
    info_i[0] = info_i[1] = info_i[3] = 0;
    info_i[2] = OR_EINVAL;
    info_d[0] = info_d[1] = info_d[2] = info_d[3] = 0.0;
    if (n <= 0 || m <= 0 || max_iters < 0 || !(rtol >= 0.0) || rmax < 0) return OR_EINVAL;
    if (!finite_all(rowptr[n], vals) || !finite_all(n, b) || (x0 && !finite_all(n, x0))) {
        info_i[2] = OR_ENONFINITE;
        return OR_ENONFINITE;
    }
    int st = OR_OK;
    adapt_state a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.rmax = rmax;
    const int32_t ld = rmax + 1;
    a.U = (double *)calloc((size_t)n * ld, sizeof(double));
    a.AU = (double *)calloc((size_t)n * ld, sizeof(double));
    a.T = (double *)calloc((size_t)ld * ld, sizeof(double));
    a.C = (double *)calloc((size_t)ld * ld, sizeof(double));
    a.t = (double *)calloc((size_t)ld, sizeof(double));
    a.s = (double *)calloc((size_t)ld, sizeof(double));
    double *V = (double *)calloc((size_t)n * (m + 1), sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));   /* rotated */
    double *H0 = (double *)calloc((size_t)(m + 1) * m, sizeof(double));  /* unrotated */
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *yv = (double *)calloc((size_t)m, sizeof(double));
    double *rv = (double *)calloc((size_t)n, sizeof(double));
    double *tmp = (double *)calloc((size_t)n, sizeof(double));
    double *d = (double *)calloc((size_t)n, sizeof(double));
    if (!a.U || !a.AU || !a.T || !a.C || !a.t || !a.s || !V || !H || !H0 || !cs || !sn || !g ||
        !yv || !rv || !tmp || !d) {
        st = OR_ENOMEM;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) x[i] = x0 ? x0[i] : 0.0;
    oracle_spmv(n, rowptr, colind, vals, x, tmp);
    for (int64_t i = 0; i < n; ++i) rv[i] = b[i] - tmp[i];
    const double rho0 = oracle_nrm2(n, rv);
    info_d[0] = rho0;
    if (rho0 == 0.0) goto done;
    const double target = rtol * rho0;
    int64_t its = 0, cycles = 0;
    double beta = rho0;
    for (;;) {
        oracle_spmv(n, rowptr, colind, vals, x, tmp);
        for (int64_t i = 0; i < n; ++i) rv[i] = b[i] - tmp[i];
        beta = oracle_nrm2(n, rv);
        if (beta <= target) { st = OR_OK; break; }
        if (its >= max_iters) { st = OR_MAXITER; break; }
        ++cycles;
        for (int64_t i = 0; i < n; ++i) V[i] = rv[i] / beta;   /* v1 = r / beta */
        for (int32_t i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int32_t k = 0;
        for (int32_t j = 0; j < m && its < max_iters; ++j) {
            const double *vj = V + (size_t)j * n;
            double *w = V + (size_t)(j + 1) * n;
            apply_minv(&a, vj, d);                        /* d = M^{-1} v_j */
            oracle_spmv(n, rowptr, colind, vals, d, w);    /* w = A M^{-1} v_j */
            ++its;
            const double wpre = oracle_nrm2(n, w);
            for (int32_t i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * n;
                const double hij = oracle_dot(n, vi, w);
                H[(int64_t)i * m + j] = hij;
                H0[(int64_t)i * m + j] = hij;
                for (int64_t q = 0; q < n; ++q) w[q] -= hij * vi[q];
            }
            const double hn = oracle_nrm2(n, w);
            H[(int64_t)(j + 1) * m + j] = hn;
            H0[(int64_t)(j + 1) * m + j] = hn;
            const int breakdown = !(hn > DBL_EPSILON * wpre);
            if (!breakdown)
                for (int64_t q = 0; q < n; ++q) w[q] /= hn;
            for (int32_t i = 0; i < j; ++i) {
                const double aa = H[(int64_t)i * m + j], cc = H[(int64_t)(i + 1) * m + j];
                H[(int64_t)i * m + j] = cs[i] * aa + sn[i] * cc;
                H[(int64_t)(i + 1) * m + j] = -sn[i] * aa + cs[i] * cc;
            }
            const double aa = H[(int64_t)j * m + j], cc = H[(int64_t)(j + 1) * m + j];
            double rho = hypot(aa, cc);
            if (cc == 0.0) { cs[j] = 1.0; sn[j] = 0.0; rho = aa; }
            else { cs[j] = aa / rho; sn[j] = cc / rho; }
            H[(int64_t)j * m + j] = rho;
            H[(int64_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            if (hist) hist[its - 1] = fabs(g[j + 1]);
            k = j + 1;
            if (fabs(g[j + 1]) <= target || breakdown) break;
        }
        for (int32_t i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int32_t q = i + 1; q < k; ++q) s -= H[(int64_t)i * m + q] * yv[q];
            yv[i] = s / H[(int64_t)i * m + i];
        }
        memset(d, 0, sizeof(double) * (size_t)n);
        for (int32_t i = 0; i < k; ++i) {
            const double *vi = V + (size_t)i * n;
            for (int64_t q = 0; q < n; ++q) d[q] += yv[i] * vi[q];
        }
        apply_minv(&a, d, d);                              /* x += M^{-1} V_k y_k */
        for (int64_t q = 0; q < n; ++q) x[q] += d[q];
        if (rmax > 0) adapt(&a, n, rowptr, colind, vals, V, H0, m, k);
    }
    info_i[0] = its;
    info_i[1] = cycles;
    info_d[1] = beta / rho0;
    oracle_spmv(n, rowptr, colind, vals, x, tmp);
    for (int64_t i = 0; i < n; ++i) tmp[i] = b[i] - tmp[i];
    info_d[2] = oracle_nrm2(n, tmp) / rho0;
    info_d[3] = a.mu;
done:
    info_i[2] = st;
    info_i[3] = a.r;
    if (st == OR_OK || st == OR_MAXITER) {
        if (Uout && rmax > 0) memcpy(Uout, a.U, sizeof(double) * (size_t)n * a.r);
        if (Tout && rmax > 0)
            for (int32_t i = 0; i < a.r; ++i)
                for (int32_t q = 0; q < a.r; ++q) Tout[(int64_t)i * a.r + q] = a.T[(int64_t)i * ld + q];
    }
    free(a.U); free(a.AU); free(a.T); free(a.C); free(a.t); free(a.s);
    free(V); free(H); free(H0); free(cs); free(sn); free(g); free(yv); free(rv); free(tmp); free(d);
    return st;
}
