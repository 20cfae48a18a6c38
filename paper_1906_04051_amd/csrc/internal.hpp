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
constexpr int kStatusNoMem = -5;      // workspace too small (gmres_status EWORKSPACE)
constexpr int kStatusHandoff = 100;   // batched: the system continues on its attached plan (internal)

// Device memory carved out of one caller-owned workspace: persistent buffers
// grow from the bottom, the temporaries of a setup step from the top (given
// back with release(mark)).  Nothing is allocated.  A request that does not
// fit returns nullptr and sets `short_`; `peak` is the largest extent any
// request reached (what the workspace would have needed so far).  With
// sizing = true no memory stands behind the arena: requests always succeed,
// the returned addresses are not usable, and `peak` measures a layout.
struct Arena {
    uintptr_t base = 0;
    size_t cap = 0, lo = 0, hi = 0, peak = 0;
    bool sizing = false;
    bool short_ = false;
    static size_t round(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); }
    void* take(size_t bytes) {
        bytes = round(bytes);
        peak = std::max(peak, lo + bytes + hi);
        if (!sizing && lo + bytes + hi > cap) {
            short_ = true;
            return nullptr;
        }
        void* q = reinterpret_cast<void*>(base + lo);
        lo += bytes;
        return q;
    }
    void* temp(size_t bytes) {
        bytes = round(bytes);
        peak = std::max(peak, lo + hi + bytes);
        if (!sizing && lo + hi + bytes > cap) {
            short_ = true;
            return nullptr;
        }
        hi += bytes;
        return reinterpret_cast<void*>(base + cap - hi);
    }
    template <typename T>
    T* take_n(int64_t count) { return static_cast<T*>(take((size_t)std::max<int64_t>(count, 1) * sizeof(T))); }
    template <typename T>
    T* temp_n(int64_t count) { return static_cast<T*>(temp((size_t)std::max<int64_t>(count, 1) * sizeof(T))); }
    size_t mark() const { return hi; }
    void release(size_t m) { hi = m; }
};

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
void launch_ctrl_reset(hipStream_t st, Ctrl* c, int64_t max_iters, int64_t hist_base);
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
// Exclusive scan of count ints into out (out[count] is not written); temps
// from `ar`; *total (host) = the int64 sum of all inputs.  The int32 outputs
// are meaningful only when *total < 2^31.
int scan_i32(hipStream_t st, Arena& ar, const int* in, int* out, int64_t count, int64_t* total);
// CSR transpose (stable: rows of the transpose in increasing original row);
// tperm[q] = original entry of transposed entry q.  Temporaries from `ar`.
int build_transpose(hipStream_t st, Arena& ar, int64_t nrows, int64_t ncols, int64_t nnz,
                    const int* rowptr, const int* colind, int* trowptr, int* tcolind, int* tperm);
size_t transpose_temp_bytes(int64_t ncols, int64_t nnz);
void gather_values(hipStream_t st, int64_t nnz, const int* perm, const double* src, double* dst);
// Row pointer of the compact A Z (n + 1) and its entry count; kStatusInval
// when a row reaches more than kAzRowMax deflation columns.
int az_count(const SetupArgs& a, Arena& ar, const int* rowptr, const int* colind, int* az_rowptr,
             int64_t* az_nnz, int* d_flags);
size_t az_count_temp_bytes(int64_t n);
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
// Sliced ELL (64-row slices, rows optionally sorted within 256-row blocks).
// sell_plan: slice offsets into off (nsl + 1 ints), the sorted row order into
// perm (n ints) and *sorted = whether it is kept, the entry count *total
// (padding included) and *wuni (uniform width, 0 if not).  *usable = false
// when the copy would hold more than `budget` entries or 2^31 or more (the
// plan then uses the CSR kernels).
int sell_plan(hipStream_t st, Arena& ar, int64_t n, const int* rowptr, int* off, int* perm,
              int64_t budget, bool* usable, bool* sorted, int64_t* total, int* wuni);
size_t sell_plan_temp_bytes(int64_t n);
// Column offsets and source entries of the planned copy; *usable = false when
// an offset col - row falls outside [-32767, 32767].
int sell_fill_pattern(hipStream_t st, int64_t n, const int* rowptr, const int* colind, const int* off,
                      const int* perm, short* scol, int* src, int* d_flags, bool* usable);
void sell_values(hipStream_t st, int64_t total, const int* src, const double* vals, double* v64,
                 float* v32);
// Single-entry row copies of a CSR (see setup.hip); c1 may be NULL (values only).
void ell1_build(hipStream_t st, int64_t n, const int* rp, const int* ci, const double* v, int* c1,
                double* v1, float* v1f);
void ell2_build(hipStream_t st, int64_t n, const int* rp, const int* ci, const double* v, int* c2,
                double* v2, float* v2f);
void invperm(hipStream_t st, int64_t m, const int* perm, int* pos);
// Per-block deflation slots for the fused Z^T y (see setup.hip) into
// caller-provided buffers: bb_ptr (nblk + 1), bb_col and ab_slot (cap each),
// ab_ptr (R + 1).  kStatusInval: some row block reaches more than
// kBlockColsMax columns, or more than cap slots are needed (the plan then
// keeps the separate Z^T pass).
int build_block_slots(hipStream_t st, Arena& ar, int64_t n, int RB, int R, const int* zrp,
                      const int* zci, int* bb_ptr, int* bb_col, int* ab_ptr, int* ab_slot,
                      int64_t cap, int64_t* nslots, int* d_flags);
size_t block_slots_temp_bytes(int64_t n, int RB, int R, int64_t cap);
// Upper bound of the slot count: one slot per (block, column) pair, at most
// kBlockColsMax per block, at most one per entry of Z.
inline int64_t block_slots_bound(int64_t n, int RB, int R, int64_t znnz) {
    const int64_t nblk = (n + RB - 1) / RB;
    return std::min<int64_t>(nblk * std::min<int64_t>(R, kBlockColsMax), znnz);
}

// batched.hip
// Host-visible record of a system that left the batched launch for its
// continuation plan: written before the flag, the flag last with a
// system-scope release (the system's x is in memory by then).
struct HandRec {
    int64_t its;
    double rho0;
    int32_t flag;
    int32_t pad;
};

struct BatchArgs {
    hipStream_t st;
    int nsys, m, L, wg;
    int64_t max_iters;
    double rtol;
    const int64_t *row_off, *zcol_off, *e_off, *v_off;   // device
    const int64_t* w_off;                                 // per-system work-vector regions
    const int* order;                                     // systems by decreasing work
    const int64_t* hand;   // per system: steps after which it leaves at a restart (0: never; NULL: none)
    HandRec* rec;          // per system, host-visible (pinned, coherent); NULL: none
    const int *rowptr, *colind;
    const double* vals;
    const int *azrp, *azci;
    const double* azv;
    const int *zrp, *zci;
    const double* zv;
    const int *ztrp, *ztci;
    const double* ztv;
    const int* zc1;          // Z single-entry rows (ELL-1, global rows; -2: several entries)
    const double* zv1;
    const int* az2c;         // A Z two-entry rows (ELL-2, global rows; -2: three or more)
    const double* az2v;
    // Sliced-ELL copy of the whole block-diagonal matrix in row order (NULL:
    // CSR rows): slice s holds rows 64s .. 64s + 63, column offsets col - row.
    const int* sell_off;
    int sell_wuni;           // > 0: every slice this wide (offsets computed)
    const short* sell_col;
    const double* sell_val;
    const double* Einv;
    const double *b, *x0;
    double* x;
    double* V;               // per-system basis regions ((m + 1) columns of ld = n_s rounded to even)
    double* W;               // per-system work vectors (3 of ld entries each, padding zero)
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
    // Launches after step(j) belong to block step j of the current cycle;
    // cycle_done(jd): the cycle ran jd steps (launches of later steps found
    // it ended and are not counted).
    virtual void step(int j) = 0;
    virtual void cycle_done(int jd) = 0;
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
    // Deflation basis (R = 0: none; R <= kBlockZMax): Z^T and Z (CSR), the
    // compact A Z (CSR over rows, local columns) and E^{-1} (R x R,
    // column-major: (E^{-1})_{i,a} at Einv[a R + i]).
    int R;
    const int *ztrp, *ztci;
    const double* ztv;
    const int *zrp, *zci;
    const double* zv;
    const int *azrp, *azci;
    const double* azv;
    const double* Einv;
};
constexpr int kBlockZMax = 64;   // deflation columns the block path supports
struct BlockResult {
    int64_t steps = 0;
    int cycles = 0;
    int status = 0;            // kStatusOk / MaxIter / Breakdown
    double rho0 = 0.0, rel_res_est = 0.0, rel_res_true = 0.0;
};
// Block workspace carved from caller memory of block_workspace_bytes(n, m)
// bytes (256-byte aligned).  block_bind zeroes the panels.
struct BlockWork;
size_t block_workspace_bytes(int64_t n, int m);
int block_bind(BlockWork* w, void* mem, size_t bytes, hipStream_t st, int64_t n, int m);
BlockWork* block_new();
// Static per-device scratch (block.hip): static_scratch_init looks up the
// device address of the array once per device (that device current);
// static_scratch returns it (nullptr before init) and its size.
int static_scratch_init(int device);
void* static_scratch(int device, size_t* bytes);
void block_delete(BlockWork* w);
int block_solve(BlockWork* w, const BlockArgs& a, BlockResult* res);

// Flag words of the bounds-checking build, one per translation unit (read
// and cleared; 0 in release builds).
unsigned int dbg_take_krylov();
unsigned int dbg_take_batched();
unsigned int dbg_take_block();
unsigned int dbg_take_setup();
unsigned int dbg_take_adapt();

}  // namespace gm
