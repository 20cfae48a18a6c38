// Internal declarations shared by the translation units of the library.
#pragma once

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "common.hpp"

namespace gm {

// SpMV variant code for the sliced-ELL kernel.
constexpr int kSell = -64;

// Status values (mirror gmres_status in include/gmres.h).
constexpr int kStatusOk = 0;
constexpr int kStatusMaxIter = 1;
constexpr int kStatusBreakdown = 2;
constexpr int kStatusStagnated = 3;
constexpr int kStatusInval = -1;
constexpr int kStatusSingular = -2;
constexpr int kStatusNonFinite = -3;
constexpr int kStatusDevice = -4;
constexpr int kStatusNoMem = -5;

// Precision of one solve engine.
constexpr int kPrecF64 = 0;   // FP64 values, basis, vectors and accumulation
constexpr int kPrecF32 = 1;   // FP32 values, basis, vectors and accumulation
constexpr int kPrecF16 = 2;   // FP32 values/vectors/accumulation, FP16 basis

// Hooks around the streaming kernels of a step (HIP-event timing).
// kind: 0 SpMV, 1 pass 1, 2 pass 2, 3 pass 3; j: step index in the cycle.
struct KTimer {
    virtual void begin(int kind, int j) = 0;
    virtual void end(int kind, int j) = 0;
    virtual ~KTimer() = default;
};

// Adaptive spectral deflation (the paper's M^{-1} = I + U(|mu| T^{-1} - I)U^T).
constexpr int kAdaptMax = 22;   // largest r_max

// Device-resident state of the adaptive deflation space.
struct AdaptState {
    int32_t r;        // columns of U in use
    int32_t ok;       // this restart's candidate is appended
    int32_t remove;   // this restart removes a direction
    int32_t r_old, r_new;
    int32_t pad;
    double mu;        // |mu| (largest Ritz value magnitude)
    double nu;        // norm of the orthogonalised candidate
};

struct AdaptArgs {
    int rmax;
    AdaptState* st;
    double *U, *AU;          // (rmax + 1) columns, stride ldv
    double *T, *C;           // (rmax + 1)^2 row-major, leading dimension rmax + 1
    double *s, *tcol, *trow, *hvec;   // rmax + 2 each
    double* zc;              // kMaxM Ritz coefficients on the stored basis
    double *ucand, *aucand, *dvec;    // ldv each
    double* part;            // (rmax + 2) * NB_cap partial sums
};

// Everything one solve engine needs: the operator (A or A^T), the deflation
// data, and the Krylov workspace.
struct EngineArgs {
    hipStream_t st;
    int prec;
    int n;
    double nscale;          // sqrt(n): FP16 storage scale numerator
    int L;                  // SpMV lanes per row
    int NB;                 // workgroups of the streaming kernels (partial-sum count)
    int nbcap;              // partial-sum capacity per slot (largest grid)
    int pass_grid;          // 1: Arnoldi passes run one round of resident workgroups
    int m;
    int nslot;              // index of the norm slot in `part`
    int64_t ldv;            // basis column stride (elements)
    void* V;
    void *y, *w, *p, *r;    // work vectors (type WT)
    double* xh;             // current iterate (FP64)
    const int *rowptr, *colind;
    const void* vals;       // AT
    const int *azrp, *azci; // compact A Z (CSR, n rows)
    const void* azv;        // AT
    int R, MC, CH;          // deflation count, Z^T chunks per row, chunk length
    const int *ztrp, *ztci; // Z^T (CSR, R rows)
    const double* ztv;
    double* tpart;          // R * MC partial sums of Z^T y
    const double* Einv;     // explicit E^{-1}, column-major R x R
    int trans;              // apply E^{-T} (adjoint operator)
    // Fused Z^T y in the stream SpMV (valid when fuse_rb == RB of the SpMV).
    int fuse_rb;            // 0: separate Z^T pass
    const int *zrp, *zci;   // Z (CSR, n rows)
    const double* zv;
    const int *bb_ptr, *bb_col, *ab_ptr, *slot_pos;   // slot_pos: slot -> column-contiguous position
    const int* zc1;         // Z single-entry rows (ELL-1)
    const double* zv1;
    const int* azc1;        // A Z two-entry rows (ELL-2, 2 per row, interleaved) of the operator
    const void* azv1;       // AT, 2 per row
    // Sliced ELL copy of the operator (used when L == kSell).
    const int* sell_off;
    const int* sell_perm;   // row of each position (NULL: position = row)
    int sell_wuni;          // > 0: every slice has this width (entries per row); off unused
    const short* sell_col;  // 16-bit column offsets from the row
    const void* sell_val;   // AT
    int sell_wmax;          // widest slice (entries per row)
    double *s_step, *s_res; // coarse solutions (per step / per restart)
    double* part;           // (m + 2) * NB partial sums
    double *h1, *h2, *coef1, *coef2;
    double *H, *cs, *sn, *g, *vscale;
    double *sigma, *sigma0;
    double* hist;           // optional |gamma_{k+1}| history
    int64_t hist_cap;       // entries of hist
    double* Hraw;           // optional unrotated Hessenberg of the last cycle
    Ctrl* ctrl;
    int* cyc_k;             // optional: basis size k of every cycle
    int cyc_cap;
    KTimer* timer;          // optional
    int trust_est;          // inner solves of the refinement: end on the estimate
    int lagged;             // two-pass CGS2 with lagged normalisation
    int dcgs;               // CGS2 with one reduction per step (delayed re-orthogonalisation)
    int cache_cols;         // FP64 basis: leading columns kept in the last-level cache
    int sell_stream;        // the sliced-ELL matrix streams past that cache (chunked rows)
    double* dcs;            // its slot sums (2m + 3)
    const AdaptArgs* adapt; // FP64 adaptive spectral deflation (nullptr: off)
    double* cc;             // lagged: coefficients (Hbar h2) of the next step, m + 1
    double* lag;            // lagged: h2_last, 1/hn, sigma
};

// adapt.hip
void adapt_reset(hipStream_t st, const AdaptArgs& a);
void adapt_pre(const EngineArgs& e, const double* x, const double* scale);
void adapt_post(const EngineArgs& e, double* y);
void adapt_cycle_end(const EngineArgs& e, const double* V, const double* coef);

// krylov.hip
// Timing events for the next timed launch of the engine on this thread
// (start / end of that kernel's execution); disarm returns true when the
// armed pair was not consumed by a launch.
void arm_kernel_events(hipEvent_t start, hipEvent_t stop);
bool disarm_kernel_events();
// Takes the armed event pair (if any) for a launch made outside krylov.hip.
bool take_kernel_events(hipEvent_t* start, hipEvent_t* stop);
void launch_restart_init(const EngineArgs& a, const void* b, double rtol, double r0_override);
void launch_cycle(const EngineArgs& a, const void* b);
void launch_correct(hipStream_t st, int NB, int n, const int* zrp, const int* zci, const double* zv,
                    const double* s, int R, const double* xh, double* x);
void launch_residual_f64(hipStream_t st, int L, int NB, int n, const int* rp, const int* ci,
                         const double* v, const double* x, const double* b, double* r, double* part,
                         int slot);
void launch_sum_slot(hipStream_t st, const double* part, int NB, int slot, double* out);
void launch_spmv_f64(hipStream_t st, int L, int NB, int n, const int* rp, const int* ci,
                     const double* v, const double* x, double* y);
void launch_spmv_sell_f64(hipStream_t st, int NB, int n, const int* off, const int* perm, int wuni,
                          int wmax, const short* col, const double* val, const double* x, double* y);
void launch_residual_sell_f64(hipStream_t st, int NB, int n, const int* off, const int* perm,
                              int wuni, int wmax, const short* col, const double* val, const double* x,
                              const double* b, double* r, double* part, int slot);
void launch_spmv_f32(hipStream_t st, int L, int NB, int n, const int* rp, const int* ci,
                     const float* v, const float* x, float* y);
void launch_scale_to_f32(hipStream_t st, int NB, int n, const double* r, const double* nrm2,
                         float* out);
void launch_axpy_norm(hipStream_t st, int NB, int n, const double* nrm2, const double* d, double* x);
void launch_ctrl_reset(hipStream_t st, Ctrl* c, int64_t max_iters);
void launch_fill(hipStream_t st, double* p, int64_t n, double v);
void launch_copy(hipStream_t st, const double* a, double* b, int64_t n);

// setup.hip
struct SetupArgs {
    hipStream_t st;
    int nsys;
    int64_t n, nnz, znnz;
    int R;                                   // total deflation columns
    const int64_t* d_sys_row_off;            // device copies, nsys + 1
    const int64_t* d_sys_zcol_off;
    const int *rowptr, *colind;
    const double* vals;
    const int *zrp, *zci;
    const double* zv;
};
int setup_validate(const SetupArgs& a, int* d_flags);       // returns a status
int build_transpose(hipStream_t st, int64_t nrows, int64_t ncols, int64_t nnz, const int* rowptr,
                    const int* colind, int* trowptr, int* tcolind, int* tperm);
void gather_values(hipStream_t st, int64_t nnz, const int* perm, const double* src, double* dst);
int az_count(const SetupArgs& a, const int* rowptr, const int* colind, int* az_rowptr,
             int64_t* az_nnz);
void az_fill(const SetupArgs& a, const int* rowptr, const int* colind, const double* vals,
             const int* az_rowptr, int* az_colind, double* az_vals);
void build_coarse(const SetupArgs& a, const int* ztrp, const int* ztci, const double* ztv,
                  const int* azrp, const int* azci, const double* azv, const int64_t* d_e_off,
                  double* E);
int lu_inverse(hipStream_t st, int nsys, const int64_t* d_sys_zcol_off, const int64_t* d_e_off,
               double* E, double* Einv, int* d_flags);
void to_f32(hipStream_t st, int64_t n, const double* src, float* dst);
void grad_vals(hipStream_t st, int64_t n, const int* rowptr, const int* colind, const double* lam,
               const double* x, double* g);
int zt_max_row(hipStream_t st, int R, const int* ztrp, int* d_tmp);
// Sliced ELL (64-row slices, rows optionally sorted within 256-row blocks;
// *perm NULL when not) of a CSR matrix; buffers hipMalloc'ed here.
int sell_build(hipStream_t st, int64_t n, const int* rowptr, const int* colind, int** off,
               int** perm, short** scol, int** src, int64_t* total, int* wuni);
void sell_values(hipStream_t st, int64_t total, const int* src, const double* vals, double* v64,
                 float* v32);
// Single-entry row copies of a CSR (see setup.hip); c1 may be NULL (values only).
void ell1_build(hipStream_t st, int64_t n, const int* rp, const int* ci, const double* v, int* c1,
                double* v1, float* v1f);
void ell2_build(hipStream_t st, int64_t n, const int* rp, const int* ci, const double* v, int* c2,
                double* v2, float* v2f);
void invperm(hipStream_t st, int64_t m, const int* perm, int* pos);
// Per-block deflation slots for the fused Z^T y (see setup.hip).  Buffers are
// hipMalloc'ed here; the caller owns them.
int build_block_slots(hipStream_t st, int64_t n, int RB, int R, const int* zrp, const int* zci,
                      int** bb_ptr, int** bb_col, int** ab_ptr, int** ab_slot, int64_t* nslots,
                      int* d_flags);

// batched.hip
struct BatchArgs {
    hipStream_t st;
    int nsys, m, L, wg;
    int64_t max_iters;
    double rtol;
    const int64_t *row_off, *zcol_off, *e_off, *v_off;   // device
    const int* order;                                     // systems by decreasing work
    const int *rowptr, *colind;
    const double* vals;
    const int *azrp, *azci;
    const double* azv;
    const int *zrp, *zci;
    const double* zv;
    const int *ztrp, *ztci;
    const double* ztv;
    const double* Einv;
    const double *b, *x0;
    double* x;
    double* V;               // per-system basis regions
    double* W;               // per-system work vectors (3 per row)
    double* small;           // per-system small state
    int64_t small_stride;
    int* ticket;
    int64_t* out_i;          // per system: its, cycles, status
    double* out_d;           // per system: rho0, rel_res, t_start, t_end
};
void launch_batched(const BatchArgs& a, int nwg);
void launch_seg_resid(hipStream_t st, int nsys, const int64_t* row_off, const int* rowptr,
                      const int* colind, const double* vals, const double* x, const double* b,
                      double* out);
// One launch of a pass kernel (FP64) for tuning: kind 1, 2 or 3 at nv columns.
void launch_pass_probe(const EngineArgs& a, int kind, int nv);


// ---------------------------------------------------------------- block GMRES
// Block GMRES(m) for k <= 16 right-hand sides (block.hip).
constexpr int kBlockStepsMax = 16;   // block steps per cycle
// Per-launch timing of the block kernels: begin() may arm events that the
// next launch carries (kinds 5 dots, 6 panel products, 7 SpMM; bytes =
// algorithmic bytes of the launch).
struct BlockTimer {
    virtual void begin(int kind, double bytes) = 0;
    virtual void end() = 0;
    virtual ~BlockTimer() = default;
};
struct BlockArgs {
    hipStream_t st;
    const int* rowptr;
    const int* colind;
    const double* vals;
    int k, m;                  // right-hand sides, block steps per cycle
    double rtol;
    int64_t max_steps;         // block steps over all cycles
    const double* B;           // n x k row-major (device)
    const double* X0;          // n x k row-major or NULL (zero)
    double* X;                 // n x k row-major (device, output)
    int64_t nnz;
    BlockTimer* timer;         // NULL: untimed
};
struct BlockResult {
    int64_t steps = 0;
    int cycles = 0;
    int status = 0;            // kStatusOk / MaxIter / Breakdown
    double rho0 = 0.0, rel_res_est = 0.0, rel_res_true = 0.0;
};
struct BlockWork;
int block_alloc(BlockWork** out, hipStream_t st, int64_t n, int m);
void block_free(BlockWork* w);
int block_solve(BlockWork* w, const BlockArgs& a, BlockResult* res);

}  // namespace gm
