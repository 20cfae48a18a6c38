/*
 * gmres.h -- C interface of the MI355X (gfx950) deflated GMRES(m) library.
 *
 * The solver computes x with A x = b by restarted GMRES(m) (arXiv 1906.04051,
 * Sec. 3.2: Arnoldi basis of the Krylov space, eq. krylov-basis; least squares
 * with the Hessenberg matrix reduced by plane rotations, eqs. arg and
 * hessenberg; residual estimate |gamma_{k+1}|, eq. res; restarts from x_m;
 * termination on ||b - A x|| / ||b - A x0|| <= rtol, eq. relative) applied to
 * the deflated operator P A, P = I - A Z E^{-1} Z^T with E = Z^T A Z for a
 * caller-supplied basis Z (the role of U and T_r = U^T A U in Sec. 3.3,
 * eqs. precond2 and tau_mat).  The returned solution carries the coarse
 * correction x = x_hat + Z E^{-1} Z^T (b - A x_hat), so b - A x = P (b - A x_hat)
 * and the stopping test is on the true residual of x.
 *
 * Conventions for every function:
 *   - Pointers without the suffix _h are DEVICE pointers (hipMalloc / torch
 *     CUDA tensors) of the device current when gmres_setup was called; _h
 *     pointers are host memory.
 *   - Matrices are CSR with int32 row pointers and column indices (0-based)
 *     and float64 values (Sec. 4: CSR storage, double precision).
 *   - Functions return a gmres_status: negative values are errors (outputs are
 *     untouched unless stated), positive values are non-fatal outcomes.  The
 *     message of the last error on the calling thread is gmres_last_error().
 *   - All device work is enqueued on the plan's stream; functions that report
 *     results on the host synchronise that stream before returning.
 *   - No function aborts, throws or prints.
 */
#ifndef GMRES_MI355X_H
#define GMRES_MI355X_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmres_plan_s* gmres_plan;

typedef enum {
    GMRES_OK = 0,           /* converged: ||b - A x|| <= rtol * ||b - A x0|| */
    GMRES_MAXITER = 1,      /* iteration cap reached; x holds the last iterate (with rtol = 0
                               this is the normal end of the fixed-count protocol, Sec. 4) */
    GMRES_BREAKDOWN = 2,    /* reserved: breakdowns are resolved by the true-residual test */
    GMRES_STAGNATED = 3,    /* mixed precision: refinement stopped reducing the FP64 residual */
    GMRES_EINVAL = -1,      /* invalid argument or malformed CSR */
    GMRES_ESINGULAR = -2,   /* E = Z^T A Z is singular (|pivot| <= r * eps * max|E|) */
    GMRES_ENONFINITE = -3,  /* NaN or Inf in A, Z, b or x0 */
    GMRES_EDEVICE = -4,     /* HIP runtime error */
    GMRES_EWORKSPACE = -5   /* the caller's workspace is too small (gmres_workspace_required) */
} gmres_status;

typedef enum {
    GMRES_FP64 = 0,          /* FP64 values, basis, vectors and reductions */
    GMRES_MIXED_F32 = 1,     /* FP64 iterative refinement around an FP32 inner solve (FP32 basis) */
    GMRES_MIXED_F16 = 2      /* as above with an FP16-stored basis (per-vector scale) */
} gmres_precision;

typedef struct {
    int32_t m;                /* restart length, 1 <= m <= 96 (Sec. 3.2, GMRES(m)) */
    int64_t max_iters;        /* cap on inner Arnoldi steps over all restarts (FP64 path) */
    double  rtol;             /* relative tolerance on ||b - A x||; 0 = run exactly max_iters
                                 steps (the paper's fixed-count protocol, Sec. 4) */
    double  r0_norm_override; /* > 0: use as ||b - A x0|| (resume from a checkpointed x) */
    int32_t precision;        /* gmres_precision */
    double  inner_rtol;       /* mixed: tightest relative tolerance of an inner solve; the
                                 reduction still needed (margin 2) is split evenly over the
                                 fewest inner solves no tighter than this */
    int32_t max_refine;       /* mixed: cap on refinement steps */
    int64_t inner_max_iters;  /* mixed: cap on inner steps per refinement */
    int32_t use_graph;        /* 1: replay each restart cycle as a captured hipGraph */
    int32_t record_history;   /* 1: keep |gamma_{k+1}| per step (gmres_history) */
    int32_t spmv_lanes;       /* SpMV variant: lanes per CSR row (1..64, power of two), or
                                 -256 / -128 for the LDS-staged row stream with that many
                                 rows per workgroup; 0 = auto */
    int32_t num_blocks;       /* workgroups of the streaming kernels; 0 = auto */
    int32_t batch_wg;         /* batched: threads per workgroup (256, 512, 1024); 0 = auto */
    int32_t batch_lanes;      /* batched: SpMV lanes per row (4, 8, 16, 32); 0 = auto */
    int32_t ortho;            /* single-system Arnoldi: 0 = CGS2 in three sweeps over the basis
                                 (project, re-project, update); 1 = CGS2 in two sweeps with lagged
                                 normalisation (the SpMV of step j+1 runs on the once-projected
                                 vector; the second update is folded into the next sweep through
                                 the Arnoldi relation); 2 = CGS2 with one reduction per step
                                 (delayed re-orthogonalisation: one dot sweep of q and A q against
                                 the basis, one update sweep; FP64 single-system plans without
                                 adaptive deflation).  Equal in exact arithmetic. */
    int32_t adapt_rmax;       /* > 0: right preconditioning by the paper's adaptive spectral
                                 deflation M^{-1} = I + U (|mu| T^{-1} - I) U^T, T = U^T A U
                                 (Sec. 3.3, eqs. precond1, precond2, tau_mat, precond3): U starts
                                 empty at every solve, gains one Ritz vector of H_k per restart
                                 (inverse iteration, u = V_k z) and keeps at most adapt_rmax
                                 columns (the direction of T's largest eigenvalue is removed);
                                 |mu| by power iteration on H_k.  1..22; needs a single-system
                                 FP64 plan, an empty Z (the fixed deflation is not combined with
                                 it) and no adjoint.  0 = off. */
} gmres_opts;

typedef struct {
    int64_t iters;            /* inner Arnoldi steps (all restarts, all refinements) */
    int32_t cycles;           /* restart cycles */
    int32_t refinements;      /* mixed: refinement steps */
    int32_t status;           /* gmres_status */
    int32_t defl_r;           /* adaptive deflation: columns of U at exit (else 0) */
    double  rho0;             /* ||b - A x0|| (or the override) */
    double  rel_res;          /* ||P (b - A x_hat)|| / rho0 at exit (= true relative residual of x) */
    double  rel_res_true;     /* ||b - A x|| / rho0 recomputed from the returned x (FP64) */
    double  solve_ms;         /* host wall time of the call */
    double  mu;               /* adaptive deflation: |mu| of the last restart (else 0) */
} gmres_info;

/* Fills *o with defaults: m = 30, max_iters = 10000, rtol = 1e-8, FP64,
 * inner_rtol = 1e-3 (FP16 basis) , max_refine = 30, inner_max_iters = 20000,
 * use_graph = 1, ortho = 1, everything else 0 (auto / off). */
void gmres_default_opts(gmres_opts* o);

/*
 * Device memory.  The library allocates none: every device buffer of a plan
 * (the copies of A and Z, Z^T, the compact A Z, E and E^{-1}, the sliced-ELL
 * and row copies, the FP32 values, A^T for the adjoint, the Krylov basis,
 * work vectors, partial sums, control block and history) is carved out of one
 * caller-owned workspace passed to gmres_setup, which must stay valid and
 * untouched until gmres_destroy.  Setup temporaries (sort and scan buffers)
 * use the top of the same workspace and are free again when setup returns.
 *
 * gmres_workspace_bytes returns the workspace size for a plan from host data
 * alone (the same sizes and options as gmres_setup; 0 for invalid arguments).
 * It is exact except for data-dependent parts, which it bounds: the compact
 * A Z (and A^T Z) gets min(n * min(r, 64), nnz * ceil(z_nnz / n)) entries --
 * an upper bound whenever every row of Z has at most ceil(z_nnz / n)
 * entries, as for indicator bases -- and the sliced-ELL copy its budget of
 * nnz + nnz/4 + 4096 entries (the plan uses the CSR kernels when the copy
 * would be larger).  When a workspace turns out too small, gmres_setup returns
 * GMRES_EWORKSPACE without touching it beyond its first workspace_bytes, and
 * gmres_workspace_required() then gives the exact size needed (call again
 * with at least that many bytes).  The workspace must be 256-byte aligned.
 */
size_t gmres_workspace_bytes(int32_t nsys, const int64_t* sys_row_off_h,
                             const int64_t* sys_zcol_off_h, int64_t nnz, int64_t z_nnz,
                             const gmres_opts* opts, int32_t need_adjoint);

/* Bytes the last GMRES_EWORKSPACE failure on the calling thread needed (0 if
 * unknown or none). */
size_t gmres_workspace_required(void);

/*
 * Builds a plan for nsys independent systems stored as one block-diagonal CSR
 * matrix of n_total = sys_row_off_h[nsys] rows (nsys = 1: a single system).
 * Rows [sys_row_off_h[s], sys_row_off_h[s+1]) form system s; their column
 * indices must lie in the same range, strictly increasing within each row
 * (sorted, no duplicates).  Z is an n_total x r_total CSR matrix (sorted
 * rows) whose columns [sys_zcol_off_h[s], sys_zcol_off_h[s+1]) belong to
 * system s (r_s = 0 allowed: plain GMRES(m)); r_s <= 256.  z_* may be NULL
 * when r_total = 0.
 *
 * Setup (Sec. 3.3 analogue, done once): validates A and Z, copies them into
 * the workspace, builds Z^T, the compact product A Z, E_s = Z^T A Z per
 * system, its LU factors with partial pivoting and the explicit inverse; for
 * need_adjoint also A^T, A^T Z and (E^T)^{-1}; FP32 copies for mixed
 * precision.  workspace / workspace_bytes: caller-owned device memory (see
 * gmres_workspace_bytes).  stream: the HIP stream for all work (0 = null
 * stream).  Errors: EINVAL (sizes, unsorted or duplicate column indices,
 * m, r_s > 256, a row of A Z with more than 64 deflation columns, a
 * misaligned workspace), ENONFINITE, ESINGULAR, EWORKSPACE, EDEVICE; *out is
 * NULL on error.
 */
gmres_status gmres_setup(gmres_plan* out, int32_t nsys, const int64_t* sys_row_off_h,
                         const int64_t* sys_zcol_off_h, const int32_t* rowptr,
                         const int32_t* colind, const double* vals, int64_t nnz,
                         const int32_t* z_rowptr, const int32_t* z_colind, const double* z_vals,
                         int64_t z_nnz, const gmres_opts* opts, int32_t need_adjoint,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Solves A x = b for a single-system plan (nsys = 1) with the plan's options
 * (FP64 or mixed-precision refinement).  b: n doubles; x0: n doubles or NULL
 * (zero initial guess, the paper's usual choice); x: n doubles (output; may
 * alias x0, not b).  info_h: optional host struct.  Returns the solve status
 * (OK, MAXITER, STAGNATED) or an error.
 */
gmres_status gmres_solve(gmres_plan p, const double* b, const double* x0, double* x,
                         gmres_info* info_h);

/*
 * Solves every system of the plan in one persistent kernel launch (FP64),
 * with a convergence state per system.  b, x0 (or NULL), x: n_total doubles
 * in the block layout of the plan.  infos_h: optional host array of nsys
 * structs (solve_ms holds that system's device solve time).  Returns OK when
 * every system converged, else the first non-OK system status.
 */
gmres_status gmres_solve_batched(gmres_plan p, const double* b, const double* x0, double* x,
                                 gmres_info* infos_h);

/*
 * Continuation plan for system s of a batched plan (nsys > 1).  In
 * gmres_solve_batched, system s leaves the persistent launch at the first
 * restart after `steps` inner steps (counted over its cycles) unless it has
 * converged, with its iterate corrected as at exit, x_s = x_hat + Z E^{-1}
 * Z^T (b_s - A x_hat); the call then continues it on `sub` -- the
 * multi-workgroup single-system engine, several such systems at a time on
 * their plans' streams -- restarted from x_s with the batch's rho0_s as the
 * tolerance reference and max_iters less the steps taken.  Restarted GMRES(m)
 * carries only the iterate from one cycle to the next (Sec. 3.2), and P A Z
 * = 0 leaves P r unchanged by the correction, so the continued solve is the
 * same iteration as staying in the batch, up to rounding.  infos_h[s] then
 * sums steps and cycles of both parts; solve_ms adds the host wall time from
 * the moment the system was seen leaving to the end of its continuation.  sub: a single-system plan (FP64 engine used whatever its
 * precision option) built on system s's rows with local indices, the same
 * values, Z columns, m and device, no adaptive deflation; it stays owned by
 * the caller and must outlive its attachment; one sub per system, and a sub
 * must not be used elsewhere while a batched solve runs.  sub = NULL
 * detaches.  gmres_update_values on the batched plan detaches every
 * continuation.  Kernel timing (gmres_set_timing) is not collected on a sub
 * while it continues a system.  The first attach allocates the plan's
 * pinned host records of the systems that leave (nsys x 24 bytes; no device
 * memory).  Errors: EINVAL (not a batched plan, s out of range, a sub of
 * another size, r or m, steps < 1, a sub already continuing another system of
 * the batch), EDEVICE.
 */
gmres_status gmres_batched_attach(gmres_plan p, int32_t s, gmres_plan sub, int64_t steps);

/*
 * Block GMRES(m_block) for k right-hand sides sharing the plan's A (several
 * right-hand sides; the paper solves one at a time, Sec. 3.2, and this is
 * the block form of the same minimisation): after j block steps of a cycle
 * X = X0 + V Y with Y minimising ||B - A X||_F over the block Krylov space
 * span{R0, A R0, ..., A^{j-1} R0}, R0 = B - A X0; cycles restart from X.
 * Single-system plans without adaptive deflation, any precision setting
 * (the solve is FP64).  With a deflation basis (R <= 64) every column is
 * deflated as in gmres_solve (Sec. 3.3): the operator is P A, R0 = P (B -
 * A X0), and at exit X = X_hat + Z E^{-1} Z^T (B - A X_hat) (eq. precond2).
 * The plan's rtol applies to every column: the solve ends when ||P (b_c -
 * A x_hat_c)|| (= ||b_c - A x_c|| after the correction; plain residuals
 * without Z) <= rtol * ||b_c - A x0_c|| for all c; max_iters caps the block
 * steps.  k in [1, 16]; m_block in [1, 16] block steps per cycle (block
 * Krylov dimension m_block * k).  B, X0 (or NULL: zero), X: n x k row-major
 * device arrays owned by the caller; X must not alias B (it may alias X0).
 * work / work_bytes: caller-owned device scratch of at least
 * gmres_block_workspace_bytes(p, m_block) bytes, 256-byte aligned ((m_block
 * + 4) panels of n x 16 doubles and the small block state); its contents
 * need not survive between calls.  info_h: iters = block steps, cycles,
 * rho0 = max_c ||b_c - A x0_c||, rel_res = max_c estimated relative residual
 * at the last block step, rel_res_true = max_c true relative residual.  Each
 * cycle runs on the columns not yet converged; a residual column that has
 * become dependent on the others adds no basis vector (the block basis may be
 * narrower than the number of right-hand sides).  Returns OK or MAXITER, or
 * EINVAL (sizes, a deflation basis of more than 64 columns, adaptive
 * deflation, a zero column of B - A X0), ENONFINITE, EWORKSPACE, EDEVICE.
 */
size_t gmres_block_workspace_bytes(gmres_plan p, int32_t m_block);
gmres_status gmres_solve_block(gmres_plan p, int32_t k, int32_t m_block, const double* B,
                               const double* X0, double* X, void* work, size_t work_bytes,
                               gmres_info* info_h);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the block
 * solve of gmres_solve_block with its scratch in a static device array of the
 * library (64 MiB per GPU, held until the process ends) instead of a caller
 * workspace.  Same arguments, results and errors as gmres_solve_block; EINVAL
 * when gmres_block_workspace_bytes(p, m_block) exceeds 64 MiB (about 65,000
 * rows at m_block = 4).  No device memory is allocated or freed.  Every call
 * on one GPU uses that GPU's array: calls that overlap on one GPU (other
 * threads, other plans, other streams) race and must be serialised by the
 * caller; the array keeps the last call's contents, and each call clears
 * what must start at zero.
 */
gmres_status gmres_solve_block_noalloc(gmres_plan p, int32_t k, int32_t m_block, const double* B,
                                       const double* X0, double* X, gmres_info* info_h);

/*
 * Adjoint of x = A^{-1} b for a single-system plan built with need_adjoint:
 * solves A^T lambda = grad_x with the same deflated GMRES(m) in FP64 (on A^T,
 * A^T Z and E^T), then grad_b = lambda and grad_vals[k] = -lambda_i x_j for
 * every stored entry k = (i, j) of A.  x: the forward solution (n doubles).
 * grad_b: n doubles; grad_vals: nnz doubles (either may be NULL to skip).
 */
gmres_status gmres_adjoint(gmres_plan p, const double* x, const double* grad_x, double* grad_b,
                           double* grad_vals, gmres_info* info_h);

/* Replaces the values of A (same pattern; nnz doubles, device) and rebuilds
 * A Z, E and its inverse, the FP32 copies and A^T's values.  ENONFINITE /
 * ESINGULAR as in setup (the plan keeps the new values either way). */
gmres_status gmres_update_values(gmres_plan p, const double* vals);

/* y = A x with the plan's FP64 SpMV kernel (n doubles each). */
gmres_status gmres_spmv(gmres_plan p, const double* x, double* y);

/* Copies min(cap, iters) entries of the |gamma_{k+1}| history of the last
 * solve (record_history = 1) to hist_h; returns the number copied or < 0. */
int64_t gmres_history(gmres_plan p, double* hist_h, int64_t cap);

/* Times candidate SpMV lane counts and streaming grid sizes on the plan's
 * matrix (and, for batches, batched workgroup shapes) with HIP events, keeps
 * the fastest in the plan, and reports them through *chosen_h (4 ints:
 * spmv_lanes, num_blocks, batch_wg, batch_lanes; may be NULL). */
gmres_status gmres_autotune(gmres_plan p, int32_t* chosen_h);

/* Per-kernel timing.  gmres_set_timing(p, period): 0 = off (the default);
 * period >= 1 = in later solves every period-th restart cycle (0, period,
 * 2*period, ...) is enqueued kernel by kernel, each timed kernel carrying a
 * pair of HIP events in its own dispatch (kernel execution time, as a kernel
 * trace reports it); the other cycles run as usual (graph replay when
 * use_graph).  EINVAL for period < 0.
 * gmres_solve_block times every launch of its dot, panel-product and SpMM
 * kernels when period >= 1.
 * gmres_kernel_times: totals over the timed cycles of the last solve (or
 * adjoint, or block solve): for kernel class k (0 SpMV, 1 first Gram-Schmidt
 * sweep, 2 second sweep, 3 third sweep of the three-sweep variant, 4 first
 * sweep of the two-sweep variant at steps j > 0, 5 block dot products
 * P^T W, 6 block panel products W +/- P C (and the sweep that applies the
 * first block projection and takes the second dot products, counted with
 * its product bytes), 7 block SpMM) writes {launches, total_ms,
 * total_algorithmic_bytes} to out_h[3*k ..]; launches that found their cycle
 * (or block cycle) already ended are not counted. */
gmres_status gmres_set_timing(gmres_plan p, int32_t period);
gmres_status gmres_kernel_times(gmres_plan p, double* out_h /* 24 doubles */);

/* Switches the stream used by later calls. */
gmres_status gmres_set_stream(gmres_plan p, hipStream_t stream);

/* Releases the plan (NULL allowed); the caller's workspace is free again afterwards. */
void gmres_destroy(gmres_plan p);

/* Message of the last error on the calling thread ("" if none). */
const char* gmres_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GMRES_MI355X_H */
