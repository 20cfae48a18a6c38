/*
 * bgmres.c -- plain FP64 CPU oracle for block GMRES(m) with k right-hand
 * sides: A X = B, X and B n x k.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library.
 *
 * The paper solves one right-hand side at a time (Sec. 3.2); several
 * right-hand sides sharing A are handled here by the block form of the same
 * minimisation.  Definition written out: after j block steps of a cycle,
 *     X = X_0 + V_j Y,   Y = argmin || B - A X ||_F,
 * over the block Krylov space span{R_0, A R_0, ..., A^{j-1} R_0} (R_0 = B - A X_0),
 * which splits into one least-squares problem per column over the same
 * space.  Built as:
 *   - V_0 S = R_0 by modified Gram-Schmidt column by column (S upper
 *     triangular, positive diagonal);
 *   - block step j: for each column c, w = A v_{jk+c} orthogonalised by
 *     modified Gram-Schmidt against every basis column so far (including the
 *     block's earlier new columns), h = coefficients, h_{(j+1)k+c, jk+c} = ||w||;
 *     this is the block Arnoldi relation A V_j = V_{j+1} Hbar_j (the analogue
 *     of eq. hessenberg) with a band Hessenberg Hbar of k subdiagonals;
 *   - the least-squares problem min || G - Hbar_j Y ||_F, G = [S; 0], by a
 *     Householder QR of Hbar_j computed from scratch after every block step;
 *     the residual of column c is the norm of the last k entries of column c
 *     of Q^T G (the analogue of eq. res);
 *   - a cycle ends when every column's estimate is <= rtol * rho0_c
 *     (rho0_c = ||b_c - A x0_c||, eq. relative per column), at m block
 *     steps, at the step cap, or at a block breakdown; X += V Y; the solve
 *     ends when every recomputed true residual passes;
 *   - a cycle runs on the columns whose true residual has not passed yet
 *     (the block shrinks as columns converge; converged columns keep x_c),
 *     since converged residuals are nearly dependent on the others.
 *
 * Readings (the GPU path uses the same ones):
 *   - iterations are counted in block steps;
 *   - block breakdown: a new column whose norm after orthogonalisation is
 *     <= BD_TOL times its norm before (the block Krylov space has stopped
 *     growing); the block step's columns of Hbar are kept, the cycle ends
 *     there (its new basis block is never used);
 *   - at a restart, a residual column dependent on the earlier ones (same
 *     test in the QR of the starting block) adds no basis vector: the cycle
 *     runs with kb <= ka basis columns per block and ka right-hand sides
 *     (G = [S; 0], S kb x ka), so restarted residuals that have become
 *     nearly dependent do not stop the solve;
 *   - a column with rho0_c = 0 is rejected (EINVAL), as is k < 1 or m < 1.
 *
 * With a deflation basis Z (r > 0), every column is deflated as in the
 * single-vector method (Sec. 3.3, eq. precond1): the operator is P A with
 * P = I - A Z E^{-1} Z^T, the starting residuals are P (b_c - A x0_c), the
 * tests compare ||P (b_c - A x_hat_c)|| with rtol * rho0_c where rho0_c =
 * ||b_c - A x0_c|| (unprojected, as for one right-hand side), and at exit
 * x_c = x_hat_c + Z E^{-1} Z^T (b_c - A x_hat_c) (eq. precond2), whose true
 * residual is P (b_c - A x_hat_c).  With k = 1 this is the deflated GMRES(m)
 * of oracle.c.
 * Build with -ffp-contract=off; sums run in index order.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BG_OK 0
#define BG_MAXITER 1
#define BG_BREAKDOWN 2
#define BG_EINVAL -1
#define BG_ENONFINITE -3
#define BG_ENOMEM -6

#define BD_TOL 1e-10

void oracle_spmv(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                 const double *x, double *y);
double oracle_dot(int64_t n, const double *a, const double *b);
double oracle_nrm2(int64_t n, const double *a);
void *oracle_defl_create(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                         int32_t r, const int32_t *zrp, const int32_t *zci, const double *zv,
                         int *status);
void oracle_defl_apply(void *d, const double *y, double *w);
void oracle_defl_correct(void *d, const double *r, double *x);
void oracle_defl_destroy(void *d);

/* Householder QR of the (rows x cols) column-major matrix M (rows >= cols),
 * applied to the (rows x k) column-major right-hand side G: on return the
 * upper triangle of M holds R and G holds Q^T G. */
static void householder_qr(int rows, int cols, double *M, int k, double *G)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)rows);
    for (int c = 0; c < cols; ++c) {
        double nrm = 0.0;
        for (int i = c; i < rows; ++i) nrm += M[(size_t)c * rows + i] * M[(size_t)c * rows + i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) continue;
        const double a0 = M[(size_t)c * rows + c];
        const double alpha = a0 >= 0.0 ? -nrm : nrm;
        for (int i = 0; i < rows; ++i) v[i] = 0.0;
        v[c] = a0 - alpha;
        for (int i = c + 1; i < rows; ++i) v[i] = M[(size_t)c * rows + i];
        double vv = 0.0;
        for (int i = c; i < rows; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        /* H = I - 2 v v^T / (v^T v) applied to the remaining columns and G. */
        for (int q = c; q < cols; ++q) {
            double s = 0.0;
            for (int i = c; i < rows; ++i) s += v[i] * M[(size_t)q * rows + i];
            s = 2.0 * s / vv;
            for (int i = c; i < rows; ++i) M[(size_t)q * rows + i] -= s * v[i];
        }
        for (int q = 0; q < k; ++q) {
            double s = 0.0;
            for (int i = c; i < rows; ++i) s += v[i] * G[(size_t)q * rows + i];
            s = 2.0 * s / vv;
            for (int i = c; i < rows; ++i) G[(size_t)q * rows + i] -= s * v[i];
        }
    }
    free(v);
}

static int finite_all(int64_t n, const double *v)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Column c of the row-major n x k matrix M into the vector out. */
static void get_col(int64_t n, int k, const double *M, int c, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = M[i * k + c];
}

/*
 * B, X0, X: n x k row-major.  max_steps caps the block steps over all cycles.
 * info_i: [block steps, cycles, -, -]; info_d: [max_c rho0_c, max_c estimated
 * relative residual at the last block step, max_c true relative residual, -].
 * hist (nullable, max_steps entries): per block step, max_c estimate / rho0_c.
 */
int oracle_bgmres(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *vals,
                  int32_t r, const int32_t *zrp, const int32_t *zci, const double *zv,
                  int32_t k, const double *B, const double *X0, int32_t m, int64_t max_steps,
                  double rtol, double *X, int64_t *info_i, double *info_d, double *hist)
{
    for (int q = 0; q < 4; ++q) {
        info_i[q] = 0;
        info_d[q] = 0.0;
    }
    if (n < 1 || k < 1 || m < 1 || max_steps < 0 || !(rtol >= 0.0) || r < 0) return BG_EINVAL;
    if (!finite_all(n * (int64_t)k, B) || !finite_all(rowptr[n], vals) ||
        (X0 && !finite_all(n * (int64_t)k, X0)))
        return BG_ENONFINITE;
    const int cols_max = m * k, rows_max = (m + 1) * k;
    double *V = (double *)calloc((size_t)rows_max * (size_t)n, sizeof(double));
    double *Hb = (double *)calloc((size_t)rows_max * (size_t)cols_max, sizeof(double)); /* col-major */
    double *M = (double *)malloc(sizeof(double) * (size_t)rows_max * (size_t)cols_max);
    double *G = (double *)malloc(sizeof(double) * (size_t)rows_max * (size_t)k);
    double *S = (double *)calloc((size_t)k * (size_t)k, sizeof(double));
    double *Y = (double *)malloc(sizeof(double) * (size_t)cols_max * (size_t)k);
    double *rho0 = (double *)malloc(sizeof(double) * (size_t)k);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *raw = (double *)malloc(sizeof(double) * (size_t)k);
    if (!V || !Hb || !M || !G || !S || !Y || !rho0 || !t || !w || !raw) {
        free(V); free(Hb); free(M); free(G); free(S); free(Y); free(rho0); free(t); free(w); free(raw);
        return BG_ENOMEM;
    }
    void *defl = NULL;
    if (r > 0) {
        int dst = 0;
        defl = oracle_defl_create(n, rowptr, colind, vals, r, zrp, zci, zv, &dst);
        if (!defl) {
            free(V); free(Hb); free(M); free(G); free(S); free(Y); free(rho0); free(t); free(w); free(raw);
            return dst == BG_ENOMEM ? BG_ENOMEM : (dst == -2 ? -2 : BG_EINVAL);
        }
    }
    for (int64_t i = 0; i < n * (int64_t)k; ++i) X[i] = X0 ? X0[i] : 0.0;

    /* R = P (B - A X) for every column, into V's first block (column
     * vectors); raw[c] = ||b_c - A x_c|| before the projection. */
#define RESIDUALS(NORMS)                                                         \
    for (int c = 0; c < k; ++c) {                                                \
        get_col(n, k, X, c, t);                                                  \
        oracle_spmv(n, rowptr, colind, vals, t, w);                              \
        for (int64_t i = 0; i < n; ++i) w[i] = B[i * k + c] - w[i];              \
        raw[c] = oracle_nrm2(n, w);                                              \
        if (defl) oracle_defl_apply(defl, w, V + (size_t)c * n);                 \
        else memcpy(V + (size_t)c * n, w, sizeof(double) * (size_t)n);           \
        NORMS[c] = oracle_nrm2(n, V + (size_t)c * n);                            \
    }

    double *rn = (double *)malloc(sizeof(double) * (size_t)k);
    int *act = (int *)malloc(sizeof(int) * (size_t)k);
    RESIDUALS(rn);
    for (int c = 0; c < k; ++c) rho0[c] = raw[c];
    double rho_max = 0.0;
    int bad = 0;
    for (int c = 0; c < k; ++c) {
        if (rho0[c] == 0.0) bad = 1;
        if (rho0[c] > rho_max) rho_max = rho0[c];
    }
    info_d[0] = rho_max;
    int status = BG_MAXITER;
    int64_t steps = 0, cycles = 0;
    double est_max = 1.0;
    if (bad) {
        status = BG_EINVAL;
        goto done;
    }
    for (;;) {
        int all = 1;
        for (int c = 0; c < k; ++c)
            if (rn[c] > rtol * rho0[c]) all = 0;
        if (all) {
            status = BG_OK;
            break;
        }
        if (steps >= max_steps) {
            status = BG_MAXITER;
            break;
        }
        /* Active columns: those whose residual has not passed yet; the cycle
         * runs on their residuals only (moved to the front of V). */
        int ka = 0;
        for (int c = 0; c < k; ++c)
            if (rn[c] > rtol * rho0[c]) {
                act[ka] = c;
                if (ka != c) memcpy(V + (size_t)ka * n, V + (size_t)c * n, sizeof(double) * (size_t)n);
                ++ka;
            }
        /* V_0 S = R by MGS over the active residual columns; a column that is
         * dependent on the accepted ones (norm after projection <= BD_TOL
         * times before) adds no basis vector but stays a right-hand side:
         * kb basis columns, ka right-hand sides, S kb x ka. */
        memset(S, 0, sizeof(double) * (size_t)k * (size_t)k);
        int kb = 0;
        for (int c = 0; c < ka; ++c) {
            memcpy(w, V + (size_t)c * n, sizeof(double) * (size_t)n);
            const double before = oracle_nrm2(n, w);
            for (int q = 0; q < kb; ++q) {
                const double h = oracle_dot(n, V + (size_t)q * n, w);
                S[(size_t)c * k + q] = h;
                for (int64_t i = 0; i < n; ++i) w[i] -= h * V[(size_t)q * n + i];
            }
            const double nv = oracle_nrm2(n, w);
            if (nv > BD_TOL * before) {
                S[(size_t)c * k + kb] = nv;
                for (int64_t i = 0; i < n; ++i) V[(size_t)kb * n + i] = w[i] / nv;
                ++kb;
            }
        }
        const int kk = kb;
        const int rmax = (m + 1) * kk;
        ++cycles;
        memset(Hb, 0, sizeof(double) * (size_t)rows_max * (size_t)cols_max);
        int j_done = 0;  /* block steps kept in this cycle */
        for (int j = 0; j < m && steps < max_steps; ++j) {
            /* Block step j: columns j kk .. j kk + kk - 1 of Hbar, basis block j+1. */
            int brk = 0;
            for (int c = 0; c < kk; ++c) {
                const int col = j * kk + c, newq = (j + 1) * kk + c;
                oracle_spmv(n, rowptr, colind, vals, V + (size_t)col * n, w);
                if (defl) {
                    oracle_defl_apply(defl, w, t);
                    memcpy(w, t, sizeof(double) * (size_t)n);
                }
                const double before = oracle_nrm2(n, w);
                for (int q = 0; q < newq; ++q) {
                    const double h = oracle_dot(n, V + (size_t)q * n, w);
                    Hb[(size_t)col * rmax + q] = h;
                    for (int64_t i = 0; i < n; ++i) w[i] -= h * V[(size_t)q * n + i];
                }
                const double hn = oracle_nrm2(n, w);
                Hb[(size_t)col * rmax + newq] = hn;
                if (!(hn > BD_TOL * before)) brk = 1;
                for (int64_t i = 0; i < n; ++i) V[(size_t)newq * n + i] = hn > 0.0 ? w[i] / hn : 0.0;
            }
            ++steps;
            j_done = j + 1;
            /* Least squares from scratch over the (j+2)kk x (j+1)kk block. */
            const int rows = (j + 2) * kk, cols = (j + 1) * kk;
            for (int q = 0; q < cols; ++q)
                for (int i = 0; i < rows; ++i) M[(size_t)q * rows + i] = Hb[(size_t)q * rmax + i];
            for (int q = 0; q < ka; ++q)
                for (int i = 0; i < rows; ++i) G[(size_t)q * rows + i] = i < kk ? S[(size_t)q * k + i] : 0.0;
            householder_qr(rows, cols, M, ka, G);
            double worst = 0.0;
            int conv = 1;
            for (int q = 0; q < ka; ++q) {
                double e = 0.0;
                for (int i = cols; i < rows; ++i) e += G[(size_t)q * rows + i] * G[(size_t)q * rows + i];
                e = sqrt(e);
                const double r0q = rho0[act[q]];
                if (e / r0q > worst) worst = e / r0q;
                if (e > rtol * r0q) conv = 0;
            }
            est_max = worst;
            if (hist) hist[steps - 1] = worst;
            if (conv || brk) break;
        }
        if (j_done > 0) {
            /* Y = R^{-1} (Q^T G)_top for the kept block steps, X += V Y. */
            const int rows = (j_done + 1) * kk, cols = j_done * kk;
            for (int q = 0; q < cols; ++q)
                for (int i = 0; i < rows; ++i) M[(size_t)q * rows + i] = Hb[(size_t)q * rmax + i];
            for (int q = 0; q < ka; ++q)
                for (int i = 0; i < rows; ++i) G[(size_t)q * rows + i] = i < kk ? S[(size_t)q * k + i] : 0.0;
            householder_qr(rows, cols, M, ka, G);
            for (int q = 0; q < ka; ++q)
                for (int i = cols - 1; i >= 0; --i) {
                    double s = G[(size_t)q * rows + i];
                    for (int l = i + 1; l < cols; ++l) s -= M[(size_t)l * rows + i] * Y[(size_t)q * cols + l];
                    Y[(size_t)q * cols + i] = s / M[(size_t)i * rows + i];
                }
            for (int64_t i = 0; i < n; ++i)
                for (int c = 0; c < ka; ++c) {
                    double s = 0.0;
                    for (int q = 0; q < cols; ++q) s += V[(size_t)q * n + i] * Y[(size_t)c * cols + q];
                    X[i * k + act[c]] += s;
                }
        }
        if (!finite_all(n * (int64_t)k, X)) {
            status = BG_ENONFINITE;
            break;
        }
        RESIDUALS(rn);
    }
done:
    if (defl && status != BG_EINVAL && status != BG_ENONFINITE) {
        /* x_c = x_hat_c + Z E^{-1} Z^T (b_c - A x_hat_c). */
        for (int c = 0; c < k; ++c) {
            get_col(n, k, X, c, t);
            oracle_spmv(n, rowptr, colind, vals, t, w);
            for (int64_t i = 0; i < n; ++i) w[i] = B[i * k + c] - w[i];
            oracle_defl_correct(defl, w, t);
            for (int64_t i = 0; i < n; ++i) X[i * k + c] = t[i];
        }
    }
    {
        double tr = 0.0;
        RESIDUALS(rn);
        for (int c = 0; c < k; ++c)
            if (rho0[c] > 0.0 && raw[c] / rho0[c] > tr) tr = raw[c] / rho0[c];
        info_d[2] = tr;
    }
    info_i[0] = steps;
    info_i[1] = cycles;
    info_d[1] = est_max;
#undef RESIDUALS
    free(V); free(Hb); free(M); free(G); free(S); free(Y); free(rho0); free(t); free(w); free(rn);
    free(act); free(raw);
    oracle_defl_destroy(defl);
    return status;
}
