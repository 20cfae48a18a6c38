// C interface of the deflated GMRES(m) library: plan setup, the host side of
// the solve loops, and the batched and adjoint entry points.
//
// The host never waits inside a restart cycle: a cycle (m Arnoldi steps, the
// end-of-cycle update and the restart decision) is enqueued as a whole --
// optionally as one captured hipGraph -- and the host reads the device control
// block of cycle c while cycle c + 1 is already queued.  One host/device
// round trip per cycle, none per step (the paper found host-side reductions
// and least squares costly, Sec. 4.4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gmres.h"
#include "internal.hpp"
#include "trace.hpp"

using namespace gm;

namespace {

thread_local std::string g_last_error;

gmres_status fail(gmres_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_OK(call)                                                                  \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess)                                                         \
            return fail(GMRES_EDEVICE, std::string(#call ": ") + hipGetErrorString(_e)); \
    } while (0)

// Algorithmic-byte accounting and HIP-event timing of the streaming kernels.
struct Timer {
    int period = 0;          // 0: off; k: time one restart cycle in k
    std::vector<hipEvent_t> pool;
    struct Rec { int kind; int cycle; int j; double bytes; int ev; };
    std::vector<Rec> recs;
    int used = 0;
    // Kernel classes: 0 SpMV, 1 first sweep, 2 second sweep, 3 third sweep
    // (three-sweep CGS2), 4 first sweep of the two-sweep variant at j > 0.
    static constexpr int kKinds = 8;
    double launches[kKinds] = {};
    double ms[kKinds] = {};
    double bytes[kKinds] = {};

    hipEvent_t ev(int i) {
        while ((int)pool.size() <= i) {
            hipEvent_t e;
            hipEventCreate(&e);
            pool.push_back(e);
        }
        return pool[i];
    }
    ~Timer() {
        for (auto e : pool) hipEventDestroy(e);
    }
    void reset() {
        recs.clear();
        used = 0;
        for (int k = 0; k < kKinds; ++k) launches[k] = ms[k] = bytes[k] = 0;
    }
};

struct Plan;

}  // namespace

struct gmres_plan_s {
    gm::BlockWork* block = nullptr;   // block GMRES buffers (bound to the caller's memory per call)
    int device = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t st = nullptr;           // plan-owned stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int nsys = 1;
    int64_t n = 0, nnz = 0, znnz = 0;
    int R = 0;
    std::vector<int64_t> row_off, zcol_off, e_off_h;
    gmres_opts o{};
    int need_adjoint = 0;
    AdaptArgs adapt{};      // adaptive spectral deflation buffers (adapt.rmax > 0)
    Arena ar;               // the caller's workspace: every device buffer of the plan
    bool sell_ok = false, tsell_ok = false;   // sliced-ELL copies planned
    bool sell_sorted = false, tsell_sorted = false;
    int64_t slots_cap = 0;  // capacity of the fused Z^T y slot lists
    int64_t mc_cap = 1;     // largest Z^T chunk count per row the partial buffer holds

    // plan-owned copies of the inputs
    int *rowptr = nullptr, *colind = nullptr;
    double* vals = nullptr;
    int *zrp = nullptr, *zci = nullptr;
    double* zv = nullptr;
    float* vals32 = nullptr;
    int64_t *d_row_off = nullptr, *d_zcol_off = nullptr, *d_e_off = nullptr;
    int* d_flags = nullptr;

    // Z^T
    int *ztrp = nullptr, *ztci = nullptr, *ztperm = nullptr;
    double* ztv = nullptr;
    int MC = 1, CH = 2048;
    // per-block deflation slots for the fused Z^T y, per stream block size
    int slots_rb = 0;
    int *bb_ptr = nullptr, *bb_col = nullptr, *ab_ptr = nullptr, *ab_slot = nullptr;
    int* slot_pos = nullptr;
    // row copies: Z single-entry (ELL-1, n rows); A Z and A^T Z two-entry
    // (ELL-2, 2 x ldv entries interleaved per row, padded)
    int* zc1 = nullptr;
    double* zv1 = nullptr;
    int *azc1 = nullptr, *atzc1 = nullptr;
    double *azv1 = nullptr, *atzv1 = nullptr;
    float* azv1f = nullptr;
    int64_t nslots = 0;
    int64_t tpart_cap = 0;
    // A Z (compact)
    int *azrp = nullptr, *azci = nullptr;
    double* azv = nullptr;
    float* azv32 = nullptr;
    int64_t az_nnz = 0;
    double *E = nullptr, *Einv = nullptr;
    // sliced ELL copies (forward op / adjoint op)
    int *sell_off = nullptr, *sell_src = nullptr;
    int *sell_perm = nullptr, *tsell_perm = nullptr;   // sorted row order (NULL: unsorted)
    short* sell_col = nullptr;   // 16-bit column offsets (NULL: no sliced ELL copy)
    double* sell_v64 = nullptr;
    float* sell_v32 = nullptr;
    int64_t sell_total = 0;
    int sell_wmax = 0, tsell_wmax = 0;
    int sell_wuni = 0, tsell_wuni = 0;   // uniform slice widths (0: not uniform)
    int *tsell_off = nullptr, *tsell_src = nullptr;
    short* tsell_col = nullptr;
    double* tsell_v64 = nullptr;
    int64_t tsell_total = 0;
    // adjoint operator
    int *trp = nullptr, *tci = nullptr, *tperm = nullptr;
    double* tv = nullptr;
    int *atzrp = nullptr, *atzci = nullptr;
    double* atzv = nullptr;
    int64_t atz_nnz = 0;

    // single-system Krylov workspace
    int NB = 1, L = 8, NB_cap = 1;
    int last_prec = 0;
    int64_t ldv = 0;
    void* V = nullptr;
    double *y = nullptr, *w = nullptr, *pv = nullptr, *rv = nullptr, *xh = nullptr, *bws = nullptr;
    double *xo = nullptr, *r64 = nullptr, *dvec = nullptr;
    double* dcs = nullptr;   // slot sums of the single-reduction CGS2 (2m + 3)
    double* part = nullptr;
    double *h1, *h2, *coef1, *coef2, *H, *Hraw, *cs, *sn, *g, *vscale, *sigma, *sigma0, *scal;
    double *cc = nullptr, *lag = nullptr;
    double *tpart = nullptr, *s_step = nullptr, *s_res = nullptr;
    Ctrl* ctrl = nullptr;
    Ctrl* ctrl_h = nullptr;             // pinned, 2 snapshots
    hipEvent_t ev_cyc[2] = {nullptr, nullptr};
    double* hist = nullptr;
    int64_t hist_cap = 0;
    int64_t hist_len = 0;
    int64_t hist_pos = 0;   // steps recorded so far by the current solve's engine runs
    int* cyc_k = nullptr;
    int64_t cyc_cap = 0;

    // graphs: [op (0 fwd, 1 adj)][prec]
    hipGraphExec_t gexec[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    hipGraph_t graph[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};

    // batched
    int batch_wg = 256, batch_L = 8;
    double *bV = nullptr, *bW = nullptr;
    double *btune_x = nullptr, *btune_b = nullptr;   // autotune: solution and right-hand side
    int* border = nullptr;
    int* bticket = nullptr;
    int64_t* bout_i = nullptr;
    double* bout_d = nullptr;
    int64_t* d_v_off = nullptr;
    int64_t* d_w_off = nullptr;
    // continuation plans of a batch (gmres_batched_attach): per system the
    // plan and the step limit after which the system leaves the batched launch
    std::vector<gmres_plan_s*> cont;
    std::vector<int64_t> cont_steps;
    int64_t* d_hand = nullptr;   // device copy of cont_steps (0: no continuation)
    int ncont = 0;
    HandRec* hrec_h = nullptr;   // pinned, coherent: systems that have left, while the launch runs
    HandRec* hrec_d = nullptr;   // the same records as the device addresses them

    Timer timer;
};

namespace {

thread_local size_t g_ws_required = 0;   // bytes the last EWORKSPACE failure needed

// Carves count elements from the plan's workspace.
template <typename T>
gmres_status dalloc(gmres_plan_s* p, T** ptr, int64_t count) {
    *ptr = p->ar.take_n<T>(count);
    if (!*ptr) return fail(GMRES_EWORKSPACE, "workspace too small");
    return GMRES_OK;
}

#define CHECK(expr)                          \
    do {                                     \
        gmres_status _s = (expr);            \
        if (_s != GMRES_OK) return _s;       \
    } while (0)

gmres_status to_status(int s, const char* what) {
    switch (s) {
        case kStatusOk: return GMRES_OK;
        case kStatusInval: return fail(GMRES_EINVAL, std::string(what) + ": invalid input");
        case kStatusSingular: return fail(GMRES_ESINGULAR, std::string(what) + ": E = Z^T A Z is singular");
        case kStatusNonFinite: return fail(GMRES_ENONFINITE, std::string(what) + ": non-finite value");
        case kStatusNoMem: return fail(GMRES_EWORKSPACE, std::string(what) + ": workspace too small");
        default: return fail(GMRES_EDEVICE, std::string(what) + ": device error");
    }
}

// SpMV variant: > 0 lanes per row; -256 / -128 LDS-staged stream with that
// many rows per block; kSell (-64) sliced ELL (short rows: FEM stencils).
// Sliced ELL for short rows, and for long rows too when its copy stores at
// most 25% padding (rows of similar length, or sorted within row blocks);
// CSR with 4 or 32 lanes per row otherwise.
int default_lanes(int64_t n, int64_t nnz, bool have_sell, int64_t sell_total) {
    const double rho = n > 0 ? (double)nnz / (double)n : 1.0;
    if (have_sell && (rho <= 40 || (double)sell_total <= 1.25 * (double)nnz)) return kSell;
    return rho <= 40 ? 4 : 32;
}

int max_row_len(hipStream_t st, int64_t n, const int* rp, int* d_tmp) {
    return zt_max_row(st, (int)n, rp, d_tmp);
}

// Single-entry (ELL-1) copies of A Z / A^T Z for the pass-1 deflation.
void refresh_ell1(gmres_plan_s* p) {
    if (p->R == 0 || !p->azc1) return;
    ell2_build(p->st, p->n, p->azrp, p->azci, p->azv, p->azc1, p->azv1, p->azv1f);
    if (p->atzc1) ell2_build(p->st, p->n, p->atzrp, p->atzci, p->atzv, p->atzc1, p->atzv1, nullptr);
}

// (Re)computes everything derived from the values of A.
gmres_status refresh_values(gmres_plan_s* p) {
    SetupArgs sa{p->st, p->nsys, p->n, p->nnz, p->znnz, p->R, p->d_row_off, p->d_zcol_off,
                 p->rowptr, p->colind, p->vals, p->zrp, p->zci, p->zv};
    if (p->R > 0) {
        az_fill(sa, p->rowptr, p->colind, p->vals, p->azrp, p->azci, p->azv);
        build_coarse(sa, p->ztrp, p->ztci, p->ztv, p->azrp, p->azci, p->azv, p->d_e_off, p->E);
        CHECK(to_status(lu_inverse(p->st, p->nsys, p->d_zcol_off, p->d_e_off, p->E, p->Einv,
                                   p->d_flags), "coarse LU"));
        if (p->azv32) to_f32(p->st, p->az_nnz, p->azv, p->azv32);
    }
    if (p->vals32) to_f32(p->st, p->nnz, p->vals, p->vals32);
    if (p->sell_src) sell_values(p->st, p->sell_total, p->sell_src, p->vals, p->sell_v64, p->sell_v32);
    if (p->need_adjoint) {
        gather_values(p->st, p->nnz, p->tperm, p->vals, p->tv);
        if (p->tsell_src) sell_values(p->st, p->tsell_total, p->tsell_src, p->tv, p->tsell_v64, nullptr);
        if (p->R > 0) az_fill(sa, p->trp, p->tci, p->tv, p->atzrp, p->atzci, p->atzv);
    }
    refresh_ell1(p);
    HIP_OK(hipStreamSynchronize(p->st));
    return GMRES_OK;
}

gmres_status clear_typed(gmres_plan_s* p);

// Row block of the stream SpMV that carries the fused Z^T y (the sliced-ELL
// kernel and the LDS-staged stream with 256 rows per workgroup).
constexpr int kSlotRB = 256;

// ------------------------------------------------------------ workspace layout
// Every device buffer of a plan is carved from the caller's workspace, in two
// phases: buffers whose sizes follow from the sizes and options (phase 1),
// then those whose sizes the setup kernels count (phase 2: the compact A Z and
// A^T Z, the sliced-ELL copies).  Setup temporaries come from the top of the
// workspace and are given back after each step: T1 while counting, T2 while
// building the fused Z^T y slots after phase 2.  The workspace needs
// P1 + max(T1, P2 + T2) bytes.

int64_t sell_budget(int64_t nnz) { return nnz + nnz / 4 + 4096; }

// Upper bound of the compact A Z entries from sizes alone: at most
// kAzRowMax per row, and at most (entries of A's row) x (entries of a Z row);
// the second factor is bounded by the mean Z row length rounded up, which is
// exact for bases with at most one entry per row (indicator bases).
int64_t az_bound(const gmres_plan_s* p) {
    if (p->R == 0 || p->n == 0) return 0;
    const int64_t zrow = std::max<int64_t>(1, (p->znnz + p->n - 1) / p->n);
    return std::min<int64_t>(p->n * std::min<int64_t>(p->R, kAzRowMax), p->nnz * zrow);
}

int64_t hist_entries(const gmres_opts& o) {
    int64_t h = o.max_iters;
    if (o.precision != GMRES_FP64) h += (int64_t)std::max(o.max_refine, 0) * std::max<int64_t>(o.inner_max_iters, 0);
    return std::min<int64_t>(std::max<int64_t>(h, 1), int64_t(1) << 24);
}

void carve_krylov(gmres_plan_s* p, Arena& A) {
    const int m = p->o.m;
    const int64_t n = p->n;
    p->ldv = (n + 63) & ~int64_t(63);
    p->V = A.take_n<double>((int64_t)(m + 1) * p->ldv);
    // Typed work vectors are read in whole 16-byte tiles: they hold ldv
    // entries and their padding stays zero.
    for (double** q : {&p->y, &p->w, &p->pv, &p->rv}) *q = A.take_n<double>(p->ldv);
    for (double** q : {&p->xh, &p->bws, &p->xo, &p->r64, &p->dvec}) *q = A.take_n<double>(n);
    p->NB_cap = std::max(p->NB, (int)std::min<int64_t>(std::max<int64_t>((n + kWG - 1) / kWG, 1), 2048));
    p->part = A.take_n<double>((int64_t)(2 * m + 3) * p->NB_cap);
    p->dcs = A.take_n<double>(2 * m + 3);
    const int64_t small = 5 * (m + 1) + 2 * (int64_t)(m + 1) * m + 2 * m + 2 * (m + 1) + 24;
    double* s = A.take_n<double>(small);
    p->h1 = s; s += m + 1;
    p->h2 = s; s += m + 1;
    p->coef1 = s; s += m + 1;
    p->coef2 = s; s += m + 1;
    p->H = s; s += (int64_t)(m + 1) * m;
    p->Hraw = s; s += (int64_t)(m + 1) * m;
    p->cs = s; s += m;
    p->sn = s; s += m;
    p->g = s; s += m + 1;
    p->vscale = s; s += m + 1;
    p->sigma = s; s += 1;
    p->sigma0 = s; s += 1;
    p->scal = s; s += 8;
    p->cc = s; s += m + 1;
    p->lag = s; s += 4;
    if (p->R > 0) {
        p->tpart_cap = std::max<int64_t>((int64_t)p->R * p->mc_cap, p->slots_cap);
        p->tpart = A.take_n<double>(p->tpart_cap);
        p->s_step = A.take_n<double>(p->R);
        p->s_res = A.take_n<double>(p->R);
        // Two entries per row (ELL-2), padded to ldv rows.
        p->azc1 = A.take_n<int>(2 * p->ldv);
        p->azv1 = A.take_n<double>(2 * p->ldv);
        if (p->o.precision != GMRES_FP64) p->azv1f = A.take_n<float>(2 * p->ldv);
        if (p->need_adjoint) {
            p->atzc1 = A.take_n<int>(2 * p->ldv);
            p->atzv1 = A.take_n<double>(2 * p->ldv);
        }
    }
    if (p->o.adapt_rmax > 0) {
        AdaptArgs& ad = p->adapt;
        const int rc = p->o.adapt_rmax + 1;
        ad.rmax = p->o.adapt_rmax;
        ad.st = A.take_n<AdaptState>(1);
        ad.U = A.take_n<double>((int64_t)rc * p->ldv);
        ad.AU = A.take_n<double>((int64_t)rc * p->ldv);
        ad.T = A.take_n<double>((int64_t)rc * rc);
        ad.C = A.take_n<double>((int64_t)rc * rc);
        for (double** q : {&ad.s, &ad.tcol, &ad.trow, &ad.hvec}) *q = A.take_n<double>(rc + 1);
        ad.zc = A.take_n<double>(kMaxM);
        for (double** q : {&ad.ucand, &ad.aucand, &ad.dvec}) *q = A.take_n<double>(p->ldv);
        ad.part = A.take_n<double>((int64_t)(rc + 1) * p->NB_cap);
    }
    p->ctrl = A.take_n<Ctrl>(1);
    p->cyc_cap = 1 << 16;
    p->cyc_k = A.take_n<int>(p->cyc_cap);
    if (p->o.record_history) {
        p->hist_cap = hist_entries(p->o);
        p->hist = A.take_n<double>(p->hist_cap);
    }
}

// Buffers of the persistent batched kernel.  A single-system plan can run it
// too (gmres_solve_batched with nsys = 1): its basis then lies in the Krylov
// basis of the plan ((m + 1) n <= (m + 1) ldv entries), which the next
// single-system solve clears again.
void carve_batched(gmres_plan_s* p, Arena& A) {
    const int ns = p->nsys;
    const int m = p->o.m;
    // Per-system regions with a leading dimension rounded up to even (16-byte
    // row pairs): at most one padding row per system.
    const int64_t padded = p->n + ns;
    if (ns > 1) {
        p->bV = A.take_n<double>((int64_t)(m + 1) * padded);
        p->btune_x = A.take_n<double>(p->n);
        p->btune_b = A.take_n<double>(p->n);
        if (p->R > 0) {
            // Two-entry row copy of A Z over the global rows.
            p->azc1 = A.take_n<int>(2 * p->n);
            p->azv1 = A.take_n<double>(2 * p->n);
        }
    } else {
        p->bV = static_cast<double*>(p->V);
    }
    p->bW = A.take_n<double>(3 * padded);
    p->d_w_off = A.take_n<int64_t>(ns);
    p->border = A.take_n<int>(ns);
    p->bticket = A.take_n<int>(1);
    p->bout_i = A.take_n<int64_t>(3 * (int64_t)ns);
    p->bout_d = A.take_n<double>(5 * (int64_t)ns);
    p->d_v_off = A.take_n<int64_t>(ns);
    if (ns > 1) p->d_hand = A.take_n<int64_t>(ns);
}

// Phase 1: buffers sized by the plan's sizes and options.
void carve_phase1(gmres_plan_s* p, Arena& A) {
    const int64_t n = p->n, nnz = p->nnz, zn = p->znnz;
    const int nsys = p->nsys;
    p->rowptr = A.take_n<int>(n + 1);
    p->colind = A.take_n<int>(nnz);
    p->vals = A.take_n<double>(nnz);
    p->d_row_off = A.take_n<int64_t>(nsys + 1);
    p->d_zcol_off = A.take_n<int64_t>(nsys + 1);
    p->d_e_off = A.take_n<int64_t>(nsys + 1);
    p->d_flags = A.take_n<int>(4);
    if (p->R > 0) {
        p->zrp = A.take_n<int>(n + 1);
        p->zci = A.take_n<int>(zn);
        p->zv = A.take_n<double>(zn);
        p->ztrp = A.take_n<int>(p->R + 1);
        p->ztci = A.take_n<int>(zn);
        p->ztperm = A.take_n<int>(zn);
        p->ztv = A.take_n<double>(zn);
        p->zc1 = A.take_n<int>(n);
        p->zv1 = A.take_n<double>(n);
        p->azrp = A.take_n<int>(n + 1);
        p->E = A.take_n<double>(p->e_off_h[nsys]);
        p->Einv = A.take_n<double>(p->e_off_h[nsys]);
        // Z^T chunk partials: at most ceil(longest Z^T row / CH) per column.
        p->mc_cap = std::max<int64_t>(1, (std::min<int64_t>(n, zn) + p->CH - 1) / p->CH);
        if (nsys == 1) {
            const int64_t nblk = (n + kSlotRB - 1) / kSlotRB;
            p->slots_cap = block_slots_bound(n, kSlotRB, p->R, zn);
            p->bb_ptr = A.take_n<int>(nblk + 1);
            p->bb_col = A.take_n<int>(p->slots_cap);
            p->ab_ptr = A.take_n<int>(p->R + 1);
            p->ab_slot = A.take_n<int>(p->slots_cap);
            p->slot_pos = A.take_n<int>(p->slots_cap);
        }
    }
    if (p->o.precision != GMRES_FP64) p->vals32 = A.take_n<float>(nnz);
    if (p->need_adjoint) {
        p->trp = A.take_n<int>(n + 1);
        p->tci = A.take_n<int>(nnz);
        p->tperm = A.take_n<int>(nnz);
        p->tv = A.take_n<double>(nnz);
        if (p->R > 0) p->atzrp = A.take_n<int>(n + 1);
    }
    const int64_t nsl = (n + 63) / 64;
    p->sell_off = A.take_n<int>(nsl + 1);
    p->sell_perm = A.take_n<int>(n);
    if (p->need_adjoint) {
        p->tsell_off = A.take_n<int>(nsl + 1);
        p->tsell_perm = A.take_n<int>(n);
    }
    if (nsys == 1) carve_krylov(p, A);
    if (p->o.m <= 64) carve_batched(p, A);
}

// Phase 2: buffers sized by the counts of the setup kernels (az_nnz,
// atz_nnz, sell_total / tsell_total with sell_ok / tsell_ok).
void carve_phase2(gmres_plan_s* p, Arena& A) {
    const bool mixed = p->o.precision != GMRES_FP64;
    if (p->R > 0) {
        p->azci = A.take_n<int>(p->az_nnz);
        p->azv = A.take_n<double>(p->az_nnz);
        if (mixed) p->azv32 = A.take_n<float>(p->az_nnz);
        if (p->need_adjoint) {
            p->atzci = A.take_n<int>(p->atz_nnz);
            p->atzv = A.take_n<double>(p->atz_nnz);
        }
    }
    if (p->sell_ok) {
        p->sell_col = A.take_n<short>(p->sell_total);
        p->sell_src = A.take_n<int>(p->sell_total);
        p->sell_v64 = A.take_n<double>(p->sell_total);
        if (mixed) p->sell_v32 = A.take_n<float>(p->sell_total);
    }
    if (p->tsell_ok) {
        p->tsell_col = A.take_n<short>(p->tsell_total);
        p->tsell_src = A.take_n<int>(p->tsell_total);
        p->tsell_v64 = A.take_n<double>(p->tsell_total);
    }
}

// Temporaries while counting (Z^T, A Z, A^T, A^T Z, sliced-ELL plans) and
// while building the fused Z^T y slots.
size_t temps_counting(const gmres_plan_s* p) {
    size_t t = sell_plan_temp_bytes(p->n);
    if (p->R > 0) t = std::max({t, transpose_temp_bytes(p->R, p->znnz), az_count_temp_bytes(p->n)});
    if (p->need_adjoint) t = std::max(t, transpose_temp_bytes(p->n, p->nnz));
    return t;
}
size_t temps_slots(const gmres_plan_s* p) {
    if (p->R == 0 || p->nsys != 1) return 0;
    return block_slots_temp_bytes(p->n, kSlotRB, p->R, p->slots_cap);
}

struct Layout {
    size_t p1 = 0, t1 = 0, p2 = 0, t2 = 0;
    size_t total() const { return p1 + std::max(t1, p2 + t2); }
};

// Sizes the layout of a plan whose size fields are set: phase 2 with the
// counts in *q when counted, else with their upper bounds.
Layout layout_of(const gmres_plan_s* q, bool counted) {
    gmres_plan_s* s = new gmres_plan_s();
    s->o = q->o;
    s->nsys = q->nsys;
    s->n = q->n;
    s->nnz = q->nnz;
    s->znnz = q->znnz;
    s->R = q->R;
    s->need_adjoint = q->need_adjoint;
    s->e_off_h = q->e_off_h;
    s->NB = q->NB;
    s->CH = q->CH;
    Arena A;
    A.sizing = true;
    Layout L;
    carve_phase1(s, A);
    L.p1 = A.lo;
    L.t1 = temps_counting(s);
    if (counted) {
        s->az_nnz = q->az_nnz;
        s->atz_nnz = q->atz_nnz;
        s->sell_ok = q->sell_ok;
        s->tsell_ok = q->tsell_ok;
        s->sell_total = q->sell_total;
        s->tsell_total = q->tsell_total;
    } else {
        s->az_nnz = s->atz_nnz = az_bound(s);
        s->sell_ok = true;
        s->tsell_ok = s->need_adjoint != 0;
        s->sell_total = s->tsell_total = sell_budget(s->nnz);
    }
    const size_t lo1 = A.lo;
    carve_phase2(s, A);
    L.p2 = A.lo - lo1;
    L.t2 = temps_slots(s);
    delete s;
    return L;
}

// Builds the per-block deflation slots used by the fused Z^T y of the stream
// SpMV (row blocks of kSlotRB rows).  Keeps the separate Z^T pass when a row
// block reaches more than 64 deflation columns.
gmres_status build_slots(gmres_plan_s* p) {
    p->slots_rb = 0;
    p->nslots = 0;
    if (p->R == 0 || p->nsys != 1 || p->slots_cap == 0) return GMRES_OK;
    int64_t ns = 0;
    const int s = build_block_slots(p->st, p->ar, p->n, kSlotRB, p->R, p->zrp, p->zci, p->bb_ptr,
                                    p->bb_col, p->ab_ptr, p->ab_slot, p->slots_cap, &ns, p->d_flags);
    if (s == kStatusInval) return GMRES_OK;          // dense Z: keep the separate pass
    CHECK(to_status(s, "deflation slots"));
    invperm(p->st, ns, p->ab_slot, p->slot_pos);
    p->nslots = ns;
    p->slots_rb = kSlotRB;
    return GMRES_OK;
}

// Zeroes and initialises the Krylov workspace; creates the host-side objects.
gmres_status init_krylov(gmres_plan_s* p) {
    CHECK(clear_typed(p));
    if (p->R > 0) {
        // Padding rows of the ELL-2 copies read as "no entry" (-1) with value 0.
        HIP_OK(hipMemsetAsync(p->azc1, 0xFF, 2 * p->ldv * sizeof(int), p->st));
        HIP_OK(hipMemsetAsync(p->azv1, 0, 2 * p->ldv * sizeof(double), p->st));
        if (p->azv1f) HIP_OK(hipMemsetAsync(p->azv1f, 0, 2 * p->ldv * sizeof(float), p->st));
        if (p->atzc1) {
            HIP_OK(hipMemsetAsync(p->atzc1, 0xFF, 2 * p->ldv * sizeof(int), p->st));
            HIP_OK(hipMemsetAsync(p->atzv1, 0, 2 * p->ldv * sizeof(double), p->st));
        }
        refresh_ell1(p);
    }
    if (p->o.adapt_rmax > 0) {
        AdaptArgs& ad = p->adapt;
        const int rc = p->o.adapt_rmax + 1;
        // Padded rows of U, AU and the candidates stay zero.
        HIP_OK(hipMemsetAsync(ad.U, 0, (size_t)rc * p->ldv * sizeof(double), p->st));
        HIP_OK(hipMemsetAsync(ad.AU, 0, (size_t)rc * p->ldv * sizeof(double), p->st));
        for (double* q : {ad.ucand, ad.aucand, ad.dvec})
            HIP_OK(hipMemsetAsync(q, 0, (size_t)p->ldv * sizeof(double), p->st));
        HIP_OK(hipMemsetAsync(ad.T, 0, (size_t)rc * rc * sizeof(double), p->st));
        HIP_OK(hipMemsetAsync(ad.C, 0, (size_t)rc * rc * sizeof(double), p->st));
    }
    HIP_OK(hipHostMalloc((void**)&p->ctrl_h, 2 * sizeof(Ctrl), 0));   // pinned host snapshots
    HIP_OK(hipEventCreateWithFlags(&p->ev_cyc[0], hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&p->ev_cyc[1], hipEventDisableTiming));
    return GMRES_OK;
}

// Zeroes the basis and the typed work vectors (their padding must read as
// zero in whichever precision the next engine uses).
gmres_status clear_typed(gmres_plan_s* p) {
    HIP_OK(hipMemsetAsync(p->V, 0, (size_t)(p->o.m + 1) * p->ldv * sizeof(double), p->st));
    for (double* q : {p->y, p->w, p->pv, p->rv})
        HIP_OK(hipMemsetAsync(q, 0, (size_t)p->ldv * sizeof(double), p->st));
    return GMRES_OK;
}

// Use of the 256 MiB last-level cache.  The matrix copy of the SpMV stays
// in it when it fits beside the work vectors one Arnoldi step touches (three
// N-vectors, with margin) and the two deflation row copies (36 B per row);
// otherwise the sliced-ELL kernel streams it (`stream`).  The leading FP64
// basis columns read with plain loads (`cols`; the rest of the basis carries
// the non-temporal hint) are as many 8N-byte columns as fill what is left of
// 94% of the cache.
struct CacheUse {
    int cols;
    int stream;
};
static CacheUse cache_use_for(const gmres_plan_s* p, int op, int prec) {
    constexpr double kUsable = 0.94 * 256.0 * 1024.0 * 1024.0;
    // Bytes per row of a work vector and of a basis column, per matrix entry.
    const double wb = (prec == kPrecF64) ? 8.0 : 4.0;
    const double vb = (prec == kPrecF64) ? 8.0 : (prec == kPrecF32 ? 4.0 : 2.0);
    const double n = (double)p->n, col = vb * n;
    double resident = 3.0 * wb * n + (p->R > 0 ? (12.0 + 3.0 * wb) * n : 0.0);
    const int64_t sell = op ? p->tsell_total : p->sell_total;
    const double mat = (p->L == kSell && sell > 0) ? (2.0 + wb) * (double)sell + 4.0 * n
                                                  : (4.0 + wb) * (double)p->nnz + 4.0 * (n + 1.0);
    const bool fits = resident + mat <= kUsable;
    if (fits) resident += mat;
    const double c = std::floor((kUsable - resident) / col);
    return {(int)std::max(0.0, std::min(c, 1024.0)), fits ? 0 : 1};
}

EngineArgs make_args(gmres_plan_s* p, int op, int prec) {
    EngineArgs a{};
    a.st = p->st;
    a.prec = prec;
    a.n = (int)p->n;
    a.nscale = std::sqrt((double)p->n);
    a.L = p->L;
    a.NB = p->NB;
    a.nbcap = p->NB_cap;
    a.pass_grid = 1;
    a.adapt = (p->adapt.rmax > 0 && op == 0 && prec == kPrecF64) ? &p->adapt : nullptr;
    a.m = p->o.m;
    a.nslot = p->o.m + 1;
    a.ldv = p->ldv;
    a.V = p->V;
    a.y = p->y;
    a.w = p->w;
    a.p = p->pv;
    a.r = p->rv;
    a.xh = p->xh;
    const bool f64 = (prec == kPrecF64);
    if (op == 0) {
        a.rowptr = p->rowptr;
        a.colind = p->colind;
        a.vals = f64 ? (const void*)p->vals : (const void*)p->vals32;
        a.azrp = p->azrp;
        a.azci = p->azci;
        a.azv = f64 ? (const void*)p->azv : (const void*)p->azv32;
        a.trans = 0;
    } else {
        a.rowptr = p->trp;
        a.colind = p->tci;
        a.vals = p->tv;
        a.azrp = p->atzrp;
        a.azci = p->atzci;
        a.azv = p->atzv;
        a.trans = 1;
    }
    a.R = p->R;
    a.MC = p->MC;
    a.CH = p->CH;
    a.ztrp = p->ztrp;
    a.ztci = p->ztci;
    a.ztv = p->ztv;
    a.tpart = p->tpart;
    a.Einv = p->Einv;
    const int rb = (p->L == kSell || p->L == -256) ? 256 : (p->L == -128 ? 128 : 0);
    a.fuse_rb = (p->R > 0 && rb != 0 && rb == p->slots_rb) ? rb : 0;
    if (op == 0) {
        a.sell_off = p->sell_off;
        a.sell_perm = p->sell_perm;
        a.sell_wuni = p->sell_wuni;
        a.sell_col = p->sell_col;
        a.sell_val = f64 ? (const void*)p->sell_v64 : (const void*)p->sell_v32;
        a.sell_wmax = p->sell_wmax;
    } else {
        a.sell_wmax = p->tsell_wmax;
        a.sell_off = p->tsell_off;
        a.sell_perm = p->tsell_perm;
        a.sell_wuni = p->tsell_wuni;
        a.sell_col = p->tsell_col;
        a.sell_val = p->tsell_v64;
    }
    a.zrp = p->zrp;
    a.zci = p->zci;
    a.zv = p->zv;
    a.bb_ptr = p->bb_ptr;
    a.bb_col = p->bb_col;
    a.ab_ptr = p->ab_ptr;
    a.slot_pos = p->slot_pos;
    a.zc1 = p->zc1;
    a.zv1 = p->zv1;
    if (op == 0) {
        a.azc1 = p->azc1;
        a.azv1 = f64 ? (const void*)p->azv1 : (const void*)p->azv1f;
    } else {
        a.azc1 = p->atzc1;
        a.azv1 = p->atzv1;
    }
    a.s_step = p->s_step;
    a.s_res = p->s_res;
    a.part = p->part;
    a.h1 = p->h1;
    a.h2 = p->h2;
    a.coef1 = p->coef1;
    a.coef2 = p->coef2;
    a.H = p->H;
    a.cs = p->cs;
    a.sn = p->sn;
    a.g = p->g;
    a.vscale = p->vscale;
    a.sigma = p->sigma;
    a.sigma0 = p->sigma0;
    a.hist = p->o.record_history ? p->hist : nullptr;
    a.hist_cap = p->hist_cap;
    a.Hraw = p->Hraw;
    a.ctrl = p->ctrl;
    a.lagged = p->o.ortho == 1 ? 1 : 0;
    a.dcgs = p->o.ortho == 2 ? 1 : 0;
    const CacheUse cu = cache_use_for(p, op, prec);
    a.cache_cols = cu.cols;
    a.sell_stream = cu.stream;
    a.dcs = p->dcs;
    a.cc = p->cc;
    a.lag = p->lag;
    a.cyc_k = p->cyc_k;
    a.cyc_cap = (int)std::min<int64_t>(p->cyc_cap, INT32_MAX);
    return a;
}

double type_bytes(int prec, int what) {
    // what: 0 matrix value, 1 basis entry, 2 work-vector entry
    if (prec == kPrecF64) return 8.0;
    if (what == 1 && prec == kPrecF16) return 2.0;
    return 4.0;
}

// Host side of the timer hooks called by the engine around streaming kernels.
struct TimerHook final : KTimer {
    gmres_plan_s* p;
    int prec;
    int op;
    int cycle = 0;
    int open_ev = -1;
    bool lagged = false, dcgs = false;
    TimerHook(gmres_plan_s* pp, int pr, int o)
        : p(pp), prec(pr), op(o), lagged(pp->o.ortho == 1), dcgs(pp->o.ortho == 2) {}
    // Algorithmic bytes of one launch: every array the kernel's scheme reads or
    // writes, touched once (cache hits not credited).  A Z is read through its
    // two-entry row copy (int32 column pairs and value pairs per row).
    double kernel_bytes(int kind, int j) const {
        const double n = (double)p->n, nnz = (double)p->nnz;
        const double bv = type_bytes(prec, 1), bw = type_bytes(prec, 2), ba = type_bytes(prec, 0);
        const double nv = j + 1;
        const double az = p->R > 0 ? (8.0 + 2.0 * ba) * n + 8.0 * p->R : 0.0;
        switch (kind) {
            case 0: {
                // Input: the stored v_0 (or v_j, three-sweep variant), else the
                // once-projected work vector.  Fused Z^T y reads Z's ELL-1 copy.
                const double bx = (!lagged || j == 0) ? bv : bw;
                const double zt = p->R > 0 ? 12.0 * n : 0.0;
                // Sliced ELL: the stored entries (value + 16-bit offset; the
                // slices' padding is not credited), slice offsets unless
                // uniform, the row order when sorted.
                const bool t = op == 1;
                const int64_t total = t ? p->tsell_total : p->sell_total;
                const int wuni = t ? p->tsell_wuni : p->sell_wuni;
                const bool sorted = (t ? p->tsell_perm : p->sell_perm) != nullptr;
                if (p->L == kSell && total > 0)
                    return (ba + 2.0) * nnz + (wuni ? 0.0 : 4.0 * (n / 64.0 + 1.0)) +
                           (sorted ? 4.0 * n : 0.0) + bx * n + bw * n + zt;
                return (ba + 4.0) * nnz + 4.0 * (n + 1) + bx * n + bw * n + zt;
            }
            case 1:
                if (dcgs && j > 0)     // reads V_0..j-1, q, y (and A Z); writes P u into y
                    return bv * n * j + bw * n + 2.0 * bw * n + az;
                if (lagged && j > 0)   // reads V_0..j-1, w1, u; writes v_j, w
                    return bv * n * (nv - 1) + bv * n + 3.0 * bw * n + az;
                return bw * n + az + bv * n * nv + bw * n;
            case 2:
                if (dcgs && j > 0)     // reads V_0..j-1, q, P u; writes v_j, w
                    return bv * n * j + 2.0 * bw * n + bv * n + bw * n;
                return bv * n * nv + 2.0 * bw * n;
            default: return bv * n * nv + bw * n + bv * n;
        }
    }
    // The events go into the dispatch of the next kernel (its own start and
    // end timestamps), not around it as markers on the stream.
    void begin(int kind, int j) override {
        Timer& t = p->timer;
        const int e0 = t.used++;
        t.used++;
        arm_kernel_events(t.ev(e0), t.ev(e0 + 1));
        const int cls = (lagged && kind == 1 && j > 0) ? 4 : kind;
        t.recs.push_back({cls, cycle, j, kernel_bytes(kind, j), e0});
    }
    void end(int, int) override {
        // A timed launch that did not go through the event-carrying path
        // leaves its record unusable.
        if (disarm_kernel_events()) p->timer.recs.back().cycle = -1;
    }
};

// Reads back the events of one engine run: launches of cycle c (in enqueue
// order) at step j did work only when j < k of device cycle c.
void collect_timer(gmres_plan_s* p, int64_t ncycles_dev) {
    Timer& t = p->timer;
    if (t.recs.empty()) return;
    std::vector<int> ks((size_t)std::max<int64_t>(ncycles_dev, 1), 0);
    const int64_t nk = std::min<int64_t>(ncycles_dev, p->cyc_cap);
    if (nk > 0) hipMemcpy(ks.data(), p->cyc_k, nk * sizeof(int), hipMemcpyDeviceToHost);
    for (const auto& r : t.recs) {
        if (r.cycle < 0 || r.cycle >= nk || r.j >= ks[r.cycle]) continue;
        float ms = 0.f;
        hipEventElapsedTime(&ms, t.pool[r.ev], t.pool[r.ev + 1]);
        t.launches[r.kind] += 1;
        t.ms[r.kind] += ms;
        t.bytes[r.kind] += r.bytes;
    }
    t.recs.clear();
    t.used = 0;
}

gmres_status ensure_graph(gmres_plan_s* p, int op, int prec, const void* b) {
    if (p->gexec[op][prec]) return GMRES_OK;
    EngineArgs a = make_args(p, op, prec);
    a.trust_est = (prec != kPrecF64) ? 1 : 0;   // reduced-precision engines only run inner solves
    hipGraph_t gph = nullptr;
    HIP_OK(hipStreamBeginCapture(p->st, hipStreamCaptureModeThreadLocal));
    launch_cycle(a, b);
    HIP_OK(hipStreamEndCapture(p->st, &gph));
    hipGraphExec_t ex = nullptr;
    HIP_OK(hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0));
    p->graph[op][prec] = gph;
    p->gexec[op][prec] = ex;
    return GMRES_OK;
}

// One run of restarted cycles of an engine from p->xh.  The host keeps two
// cycles enqueued ahead of the one whose control snapshot it reads; a cycle
// that starts after the solve has ended does nothing (device-side gate).
// Timed cycles (one in timer.period) are enqueued kernel by kernel with
// events in their timed dispatches; the others replay the cycle graph.
struct EngineRun {
    gmres_plan_s* p;
    int op, prec;
    const void* b = nullptr;
    int64_t cap = 0;
    int64_t c = 1;             // the host waits next on cycle c - 1
    bool finished = false;     // a snapshot said done
    bool exhausted = false;    // cap + 2 cycles without done
    EngineArgs a{}, at{};
    TimerHook hook;
    TraceSpan span[2];
    EngineRun(gmres_plan_s* pp, int o, int pr) : p(pp), op(o), prec(pr), hook(pp, pr, o) {}
    EngineRun(const EngineRun&) = delete;
    EngineRun& operator=(const EngineRun&) = delete;
};

gmres_status engine_enqueue(EngineRun& r, int64_t c) {
    static const char* const kCycleName[2][3] = {{"cycle fp64", "cycle fp32", "cycle fp16-basis"},
                                                 {"cycle adjoint fp64", "cycle adjoint fp32",
                                                  "cycle adjoint fp16-basis"}};
    gmres_plan_s* p = r.p;
    r.span[c & 1].start(kCycleName[r.op ? 1 : 0][r.prec]);
    const int period = p->timer.period;
    if (period > 0 && c % period == 0) {
        r.hook.cycle = (int)c;
        launch_cycle(r.at, r.b);
    } else if (p->o.use_graph != 0) {
        HIP_OK(hipGraphLaunch(p->gexec[r.op][r.prec], p->st));
    } else {
        launch_cycle(r.a, r.b);
    }
    HIP_OK(hipMemcpyAsync(&p->ctrl_h[c & 1], p->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipEventRecord(p->ev_cyc[c & 1], p->st));
    return GMRES_OK;
}

// Resets the control block, runs the restart set-up and enqueues cycles 0
// and 1.  b: the engine's right-hand side (type WT).
gmres_status engine_start(EngineRun& r, const void* b, double rtol, double r0_override, int64_t max_iters,
                          bool trust_est) {
    gmres_plan_s* p = r.p;
    r.a = make_args(p, r.op, r.prec);
    r.a.trust_est = trust_est ? 1 : 0;
    r.at = r.a;
    r.at.timer = &r.hook;
    r.b = b;
    if (p->o.use_graph != 0) CHECK(ensure_graph(p, r.op, r.prec, b));
    if (r.prec != p->last_prec) {
        CHECK(clear_typed(p));
        p->last_prec = r.prec;
    }
    launch_ctrl_reset(p->st, p->ctrl, max_iters, p->hist_pos);
    launch_restart_init(r.a, b, rtol, r0_override);
    r.cap = max_iters + 3;
    CHECK(engine_enqueue(r, 0));
    r.c = 1;
    if (r.c <= r.cap) CHECK(engine_enqueue(r, r.c));
    return GMRES_OK;
}

// Reads the snapshot of cycle c - 1 (waiting for it when block, else
// returning with *ready = false while it is still in flight); when the
// solve goes on, enqueues the next cycle.
gmres_status engine_step(EngineRun& r, bool block, bool* ready) {
    gmres_plan_s* p = r.p;
    hipEvent_t ev = p->ev_cyc[(r.c - 1) & 1];
    if (block) {
        HIP_OK(hipEventSynchronize(ev));
    } else {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();   // not an error: keep it out of the next launch check
            *ready = false;
            return GMRES_OK;
        }
        HIP_OK(e);
    }
    *ready = true;
    r.span[(r.c - 1) & 1].stop();
    if (p->ctrl_h[(r.c - 1) & 1].done) {
        r.finished = true;
        return GMRES_OK;
    }
    ++r.c;
    if (r.c > r.cap + 1) {
        r.exhausted = true;
        return GMRES_OK;
    }
    if (r.c <= r.cap) CHECK(engine_enqueue(r, r.c));
    return GMRES_OK;
}

// Waits for the plan's stream and returns the final control block in *out.
gmres_status engine_end(EngineRun& r, Ctrl* out) {
    gmres_plan_s* p = r.p;
    HIP_OK(hipStreamSynchronize(p->st));
    r.span[0].stop();
    r.span[1].stop();
    HIP_OK(hipMemcpy(out, p->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    if (p->timer.period > 0) collect_timer(p, out->cycles);
    p->hist_pos += out->its;   // the next run of the same solve records after these steps
    if (!r.finished) return fail(GMRES_EDEVICE, "solve loop did not terminate");
    return GMRES_OK;
}

// Runs restarted cycles of one engine from p->xh until the control block says
// done.  b: the engine's right-hand side (type WT).  Returns the final control
// block in *out.
gmres_status run_engine(gmres_plan_s* p, int op, int prec, const void* b, double rtol,
                        double r0_override, int64_t max_iters, Ctrl* out, bool trust_est = false) {
    EngineRun r(p, op, prec);
    CHECK(engine_start(r, b, rtol, r0_override, max_iters, trust_est));
    bool ready = false;
    while (!r.finished && !r.exhausted) CHECK(engine_step(r, true, &ready));
    return engine_end(r, out);
}

// ||b - A x|| in FP64 (scratch: p->w, partial slot of p->part).
void spmv_f64(gmres_plan_s* p, int L, int NB, const double* x, double* y) {
    if (L == kSell)
        launch_spmv_sell_f64(p->st, NB, (int)p->n, p->sell_off, p->sell_perm, p->sell_wuni, p->sell_wmax,
                             p->sell_col, p->sell_v64, x, y);
    else
        launch_spmv_f64(p->st, L, NB, (int)p->n, p->rowptr, p->colind, p->vals, x, y);
}

void residual_f64(gmres_plan_s* p, const double* x, const double* b, double* r, int slot) {
    if (p->L == kSell)
        launch_residual_sell_f64(p->st, p->NB, (int)p->n, p->sell_off, p->sell_perm, p->sell_wuni,
                                 p->sell_wmax, p->sell_col, p->sell_v64, x, b, r, p->part, slot);
    else
        launch_residual_f64(p->st, p->L, p->NB, (int)p->n, p->rowptr, p->colind, p->vals, x, b, r,
                            p->part, slot);
}

gmres_status true_residual(gmres_plan_s* p, const double* b, const double* x, double* nrm) {
    const int slot = p->o.m + 1;
    residual_f64(p, x, b, p->w, slot);
    launch_sum_slot(p->st, p->part, p->NB, slot, p->scal);
    double h = 0;
    HIP_OK(hipMemcpyAsync(&h, p->scal, sizeof(double), hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    *nrm = std::sqrt(h);
    return GMRES_OK;
}

gmres_status enter(gmres_plan_s* p) {
    HIP_OK(hipSetDevice(p->device));
    HIP_OK(hipEventRecord(p->ev_in, p->user_stream));
    HIP_OK(hipStreamWaitEvent(p->st, p->ev_in, 0));
    return GMRES_OK;
}

// Bounds-checking build: waits for the plan's stream and turns any failed
// device check into GMRES_EDEVICE.
gmres_status debug_checks(gmres_plan_s* p) {
#ifdef GMRES_DEBUG
    HIP_OK(hipStreamSynchronize(p->st));
    const unsigned int bits = dbg_take_krylov() | dbg_take_batched() | dbg_take_block() |
                              dbg_take_setup() | dbg_take_adapt();
    if (bits) {
        char msg[96];
        std::snprintf(msg, sizeof msg, "device bounds check failed (bits 0x%x)", bits);
        return fail(GMRES_EDEVICE, msg);
    }
#else
    (void)p;
#endif
    return GMRES_OK;
}

gmres_status leave(gmres_plan_s* p) {
    CHECK(debug_checks(p));
    HIP_OK(hipEventRecord(p->ev_out, p->st));
    HIP_OK(hipStreamWaitEvent(p->user_stream, p->ev_out, 0));
    return GMRES_OK;
}

// FP64 solve of op (0: A, 1: A^T) for right-hand side b (device, n) from x0
// (or zero) into x.  Fills info (iters/cycles/status/rho0/rel_res).
gmres_status solve_f64(gmres_plan_s* p, int op, const double* b, const double* x0, double* x,
                       double rtol, double r0_override, int64_t max_iters, gmres_info* info) {
    const int64_t n = p->n;
    launch_copy(p->st, b, p->bws, n);
    if (x0) launch_copy(p->st, x0, p->xh, n);
    else launch_fill(p->st, p->xh, n, 0.0);
    Ctrl c{};
    if (op == 0 && p->adapt.rmax > 0) adapt_reset(p->st, p->adapt);   // U starts empty
    CHECK(run_engine(p, op, kPrecF64, p->bws, rtol, r0_override, max_iters, &c));
    launch_correct(p->st, p->NB, (int)n, p->zrp, p->zci, p->zv, p->s_res, p->R, p->xh, x);
    if (op == 0 && p->adapt.rmax > 0) {
        AdaptState as{};
        HIP_OK(hipMemcpyAsync(&as, p->adapt.st, sizeof(as), hipMemcpyDeviceToHost, p->st));
        HIP_OK(hipStreamSynchronize(p->st));
        info->defl_r = as.r;
        info->mu = as.mu;
    }
    info->iters += c.its;
    info->cycles += c.cycles;
    info->status = c.status;
    info->rho0 = c.rho0;
    info->rel_res = c.rho0 > 0 ? c.beta / c.rho0 : 0.0;
    return GMRES_OK;
}

gmres_status solve_mixed(gmres_plan_s* p, const double* b, const double* x0, double* x,
                         gmres_info* info) {
    const int64_t n = p->n;
    const gmres_opts& o = p->o;
    const int slot = o.m + 1;
    if (x0) launch_copy(p->st, x0, p->xo, n);
    else launch_fill(p->st, p->xo, n, 0.0);
    // r = b - A x (FP64), ||r||^2 into scal[0]
    auto outer_residual = [&](double* nrm2_h) -> gmres_status {
        residual_f64(p, p->xo, b, p->r64, slot);
        launch_sum_slot(p->st, p->part, p->NB, slot, p->scal);
        HIP_OK(hipMemcpyAsync(nrm2_h, p->scal, sizeof(double), hipMemcpyDeviceToHost, p->st));
        HIP_OK(hipStreamSynchronize(p->st));
        return GMRES_OK;
    };
    double nrm2 = 0;
    CHECK(outer_residual(&nrm2));
    if (!std::isfinite(nrm2)) return fail(GMRES_ENONFINITE, "non-finite residual");
    const double rho0 = o.r0_norm_override > 0 ? o.r0_norm_override : std::sqrt(nrm2);
    const double target = o.rtol * rho0;
    info->rho0 = rho0;
    int prec = (o.precision == GMRES_MIXED_F16) ? kPrecF16 : kPrecF32;
    double rho_prev = INFINITY;
    int status = GMRES_MAXITER;
    int stalls = 0;
    for (int ref = 0;; ++ref) {
        TraceRange tr_ref("refinement");
        const double rho = std::sqrt(nrm2);
        if (rho <= target) {
            status = GMRES_OK;
            break;
        }
        if (ref >= o.max_refine) {
            status = GMRES_STAGNATED;
            break;
        }
        if (rho > 0.5 * rho_prev) {
            // No contraction: raise the inner precision (FP16 basis -> FP32
            // basis -> FP64 inner solve to the final tolerance).
            ++stalls;
            if (prec == kPrecF16) prec = kPrecF32;
            else prec = kPrecF64;
        }
        rho_prev = rho;
        if (prec == kPrecF64) {
            gmres_info sub{};
            const int64_t left = std::max<int64_t>(o.max_iters - info->iters, 1);
            CHECK(solve_f64(p, 0, b, p->xo, p->xo, o.rtol, rho0, left, &sub));
            info->iters += sub.iters;
            info->cycles += sub.cycles;
            info->refinements = ref + 1;
            CHECK(outer_residual(&nrm2));
            status = (std::sqrt(nrm2) <= target * (1 + 1e-12)) ? GMRES_OK : GMRES_STAGNATED;
            break;
        }
        // Inner solve of A d = r / ||r|| in reduced precision.  The reduction
        // still needed, with a margin of 2 (need = target / (2 rho) < 1/2), is
        // split evenly over the fewest refinements whose solves are no tighter
        // than the plan's inner tolerance: k = ceil(log need / log inner_rtol)
        // solves to need^(1/k) each.  (rtol 1e-8, inner_rtol 1e-3: three
        // solves to about 1.7e-3, where fixed 1e-3 solves overshoot; the
        // reduced-precision solves slow down near their accuracy floor.)
        const double need = 0.5 * target / rho;
        int k_left = 1;
        if (need < o.inner_rtol)
            k_left = (int)std::ceil(std::log(need) / std::log(o.inner_rtol) - 1e-9);
        const double inner =
            std::min(0.5, std::max(o.inner_rtol, std::pow(need, 1.0 / std::max(k_left, 1))));
        launch_scale_to_f32(p->st, p->NB, (int)n, p->r64, p->scal, reinterpret_cast<float*>(p->bws));
        launch_fill(p->st, p->xh, n, 0.0);
        Ctrl c{};
        CHECK(run_engine(p, 0, prec, p->bws, inner, 0.0, o.inner_max_iters, &c, true));
        launch_correct(p->st, p->NB, (int)n, p->zrp, p->zci, p->zv, p->s_res, p->R, p->xh, p->dvec);
        info->iters += c.its;
        info->cycles += c.cycles;
        info->refinements = ref + 1;
        launch_axpy_norm(p->st, p->NB, (int)n, p->scal, p->dvec, p->xo);
        CHECK(outer_residual(&nrm2));
        if (!std::isfinite(nrm2)) return fail(GMRES_ENONFINITE, "non-finite residual");
        (void)stalls;
    }
    launch_copy(p->st, p->xo, x, n);
    info->status = status;
    info->rel_res = rho0 > 0 ? std::sqrt(nrm2) / rho0 : 0.0;
    return GMRES_OK;
}

}  // namespace

// =====================================================================  C ABI

extern "C" {

void gmres_default_opts(gmres_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->m = 30;
    o->max_iters = 10000;
    o->rtol = 1e-8;
    o->precision = GMRES_FP64;
    o->inner_rtol = 1e-3;
    o->max_refine = 30;
    o->inner_max_iters = 20000;
    o->use_graph = 1;
    o->ortho = 1;
}

const char* gmres_last_error(void) { return g_last_error.c_str(); }

void gmres_destroy(gmres_plan p) {
    if (!p) return;
    hipSetDevice(p->device);
    if (p->st) hipStreamSynchronize(p->st);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            if (p->gexec[a][b]) hipGraphExecDestroy(p->gexec[a][b]);
            if (p->graph[a][b]) hipGraphDestroy(p->graph[a][b]);
        }
    gm::block_delete(p->block);
    if (p->ctrl_h) hipHostFree(p->ctrl_h);
    if (p->hrec_h) hipHostFree(p->hrec_h);
    for (auto e : {p->ev_cyc[0], p->ev_cyc[1], p->ev_in, p->ev_out})
        if (e) hipEventDestroy(e);
    if (p->st) hipStreamDestroy(p->st);
    delete p;
}

static gmres_status init_batched(gmres_plan_s* p);

// Host-side checks of the setup arguments; fills the plan's size fields.
static gmres_status check_args(gmres_plan_s* p, int32_t nsys, const int64_t* sys_row_off_h,
                               const int64_t* sys_zcol_off_h, const int32_t* rowptr,
                               const int32_t* colind, const double* vals, int64_t nnz,
                               const int32_t* z_rowptr, const int32_t* z_colind,
                               const double* z_vals, int64_t z_nnz, const gmres_opts* opts,
                               int32_t need_adjoint, bool need_arrays) {
    if (nsys < 1 || !sys_row_off_h || !opts)
        return fail(GMRES_EINVAL, "nsys, sys_row_off_h and opts are required");
    if (need_arrays && !rowptr) return fail(GMRES_EINVAL, "rowptr is required");
    p->o = *opts;
    if (p->o.m < 1 || p->o.m > kMaxM) return fail(GMRES_EINVAL, "m must be in [1, 96]");
    if (p->o.max_iters < 0 || !(p->o.rtol >= 0.0))
        return fail(GMRES_EINVAL, "max_iters >= 0 and rtol >= 0 required");
    if (p->o.precision < 0 || p->o.precision > 2) return fail(GMRES_EINVAL, "unknown precision");
    if (p->o.ortho < 0 || p->o.ortho > 2) return fail(GMRES_EINVAL, "unknown orthogonalisation variant");
    if (p->o.ortho == 2 && (p->o.precision != GMRES_FP64 || nsys != 1 || p->o.adapt_rmax > 0))
        return fail(GMRES_EINVAL, "ortho = 2 needs a single-system FP64 plan without adaptive deflation");
    if (p->o.adapt_rmax < 0 || p->o.adapt_rmax > kAdaptMax)
        return fail(GMRES_EINVAL, "adapt_rmax must be in [0, 22]");
    if (p->o.adapt_rmax > 0 && (p->o.precision != GMRES_FP64 || nsys != 1 || need_adjoint))
        return fail(GMRES_EINVAL, "adaptive deflation needs a single-system FP64 plan without adjoint");
    if (p->o.precision != GMRES_FP64 && (!(p->o.inner_rtol > 0.0) || p->o.inner_rtol >= 1.0))
        return fail(GMRES_EINVAL, "inner_rtol must be in (0, 1)");
    if (p->o.precision != GMRES_FP64 && (p->o.max_refine < 0 || p->o.inner_max_iters < 0))
        return fail(GMRES_EINVAL, "max_refine and inner_max_iters must be >= 0");
    if (p->o.num_blocks < 0 || p->o.num_blocks > 2048) return fail(GMRES_EINVAL, "num_blocks must be in [0, 2048]");
    if (p->o.spmv_lanes != 0 && p->o.spmv_lanes != -256 && p->o.spmv_lanes != -128 &&
        p->o.spmv_lanes != kSell &&
        (p->o.spmv_lanes < 1 || p->o.spmv_lanes > 64 || (p->o.spmv_lanes & (p->o.spmv_lanes - 1))))
        return fail(GMRES_EINVAL, "spmv_lanes must be a power of two in [1, 64], -64, -128 or -256");
    p->nsys = nsys;
    p->row_off.assign(sys_row_off_h, sys_row_off_h + nsys + 1);
    if (sys_zcol_off_h) p->zcol_off.assign(sys_zcol_off_h, sys_zcol_off_h + nsys + 1);
    else p->zcol_off.assign(nsys + 1, 0);
    if (p->row_off[0] != 0 || p->zcol_off[0] != 0)
        return fail(GMRES_EINVAL, "offsets must start at 0");
    for (int s = 0; s < nsys; ++s) {
        if (p->row_off[s + 1] <= p->row_off[s]) return fail(GMRES_EINVAL, "empty or negative system");
        const int64_t r = p->zcol_off[s + 1] - p->zcol_off[s];
        if (r < 0 || r > kMaxR) return fail(GMRES_EINVAL, "deflation count per system must be in [0, 256]");
        if (r > p->row_off[s + 1] - p->row_off[s])
            return fail(GMRES_EINVAL, "more deflation vectors than unknowns");
    }
    p->n = p->row_off[nsys];
    p->nnz = nnz;
    p->R = (int)p->zcol_off[nsys];
    if (p->o.adapt_rmax > 0 && p->R > 0)
        return fail(GMRES_EINVAL, "adaptive deflation is not combined with a fixed deflation basis Z");
    p->znnz = p->R > 0 ? z_nnz : 0;
    if (p->n >= INT32_MAX || nnz < 0 || nnz >= INT32_MAX || p->znnz < 0 || p->znnz >= INT32_MAX)
        return fail(GMRES_EINVAL, "sizes exceed the int32 CSR range");
    if (need_arrays && nnz > 0 && (!colind || !vals)) return fail(GMRES_EINVAL, "colind/vals required");
    if (need_arrays && p->R > 0 && (!z_rowptr || (p->znnz > 0 && (!z_colind || !z_vals))))
        return fail(GMRES_EINVAL, "Z arrays required when r > 0");
    p->need_adjoint = need_adjoint ? 1 : 0;
    if (p->need_adjoint && nsys != 1) return fail(GMRES_EINVAL, "the adjoint needs a single-system plan");
    p->e_off_h.assign(nsys + 1, 0);
    for (int s = 0; s < nsys; ++s) {
        const int64_t r = p->zcol_off[s + 1] - p->zcol_off[s];
        p->e_off_h[s + 1] = p->e_off_h[s] + r * r;
    }
    p->NB = p->o.num_blocks > 0 ? p->o.num_blocks
                                : (int)std::min<int64_t>(std::max<int64_t>((p->n + kWG - 1) / kWG, 1), 1024);
    return GMRES_OK;
}

static gmres_status short_of(size_t need) {
    g_ws_required = need;
    return fail(GMRES_EWORKSPACE, "workspace too small: " + std::to_string(need) + " bytes needed");
}

static gmres_status setup_impl(gmres_plan_s* p, int32_t nsys, const int64_t* sys_row_off_h,
                               const int64_t* sys_zcol_off_h, const int32_t* rowptr,
                               const int32_t* colind, const double* vals, int64_t nnz,
                               const int32_t* z_rowptr, const int32_t* z_colind,
                               const double* z_vals, int64_t z_nnz, const gmres_opts* opts,
                               int32_t need_adjoint, void* workspace, size_t workspace_bytes,
                               hipStream_t stream) {
    CHECK(check_args(p, nsys, sys_row_off_h, sys_zcol_off_h, rowptr, colind, vals, nnz, z_rowptr,
                     z_colind, z_vals, z_nnz, opts, need_adjoint, true));
    const Layout est = layout_of(p, false);
    if (!workspace || workspace_bytes < est.p1 + est.t1) return short_of(est.total());
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(GMRES_EINVAL, "workspace must be 256-byte aligned");
    p->ar.base = reinterpret_cast<uintptr_t>(workspace);
    p->ar.cap = workspace_bytes;

    HIP_OK(hipGetDevice(&p->device));
    // Address of the static scratch of gmres_solve_block_noalloc on this
    // device (looked up once per device; without it only that entry fails).
    if (nsys == 1) (void)gm::static_scratch_init(p->device);
    p->user_stream = stream;
    HIP_OK(hipStreamCreateWithFlags(&p->st, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
    CHECK(enter(p));

    carve_phase1(p, p->ar);
    if (p->ar.short_) return short_of(est.total());
    const size_t lo1 = p->ar.lo;

    // Plan-owned copies of A and Z.
    const int64_t n = p->n;
    HIP_OK(hipMemcpyAsync(p->rowptr, rowptr, (n + 1) * sizeof(int), hipMemcpyDeviceToDevice, p->st));
    if (nnz > 0) {
        HIP_OK(hipMemcpyAsync(p->colind, colind, nnz * sizeof(int), hipMemcpyDeviceToDevice, p->st));
        HIP_OK(hipMemcpyAsync(p->vals, vals, nnz * sizeof(double), hipMemcpyDeviceToDevice, p->st));
    }
    if (p->R > 0) {
        HIP_OK(hipMemcpyAsync(p->zrp, z_rowptr, (n + 1) * sizeof(int), hipMemcpyDeviceToDevice, p->st));
        if (p->znnz > 0) {
            HIP_OK(hipMemcpyAsync(p->zci, z_colind, p->znnz * sizeof(int), hipMemcpyDeviceToDevice, p->st));
            HIP_OK(hipMemcpyAsync(p->zv, z_vals, p->znnz * sizeof(double), hipMemcpyDeviceToDevice, p->st));
        }
    }
    HIP_OK(hipMemcpyAsync(p->d_row_off, p->row_off.data(), (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice, p->st));
    HIP_OK(hipMemcpyAsync(p->d_zcol_off, p->zcol_off.data(), (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice, p->st));
    HIP_OK(hipMemcpyAsync(p->d_e_off, p->e_off_h.data(), (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice, p->st));

    SetupArgs sa{p->st, nsys, n, nnz, p->znnz, p->R, p->d_row_off, p->d_zcol_off,
                 p->rowptr, p->colind, p->vals, p->zrp, p->zci, p->zv};
    CHECK(to_status(setup_validate(sa, p->d_flags), "input validation"));

    // Counting: Z^T, A Z, A^T, A^T Z, sliced-ELL plans (temporaries T1).
    if (p->R > 0) {
        CHECK(to_status(build_transpose(p->st, p->ar, n, p->R, p->znnz, p->zrp, p->zci, p->ztrp, p->ztci,
                                        p->ztperm), "Z transpose"));
        gather_values(p->st, p->znnz, p->ztperm, p->zv, p->ztv);
        ell1_build(p->st, n, p->zrp, p->zci, p->zv, p->zc1, p->zv1, nullptr);
        const int maxrow = zt_max_row(p->st, p->R, p->ztrp, p->d_flags);
        p->MC = std::max(1, (maxrow + p->CH - 1) / p->CH);
        const int s = az_count(sa, p->ar, p->rowptr, p->colind, p->azrp, &p->az_nnz, p->d_flags);
        if (s == kStatusInval)
            return fail(GMRES_EINVAL, "a row of A*Z reaches more than 64 deflation columns");
        CHECK(to_status(s, "A*Z"));
    }
    if (p->need_adjoint) {
        CHECK(to_status(build_transpose(p->st, p->ar, n, n, nnz, p->rowptr, p->colind, p->trp, p->tci,
                                        p->tperm), "A transpose"));
        gather_values(p->st, nnz, p->tperm, p->vals, p->tv);
        if (p->R > 0) {
            const int s = az_count(sa, p->ar, p->trp, p->tci, p->atzrp, &p->atz_nnz, p->d_flags);
            if (s == kStatusInval)
                return fail(GMRES_EINVAL, "a row of A^T*Z reaches more than 64 deflation columns");
            CHECK(to_status(s, "A^T*Z"));
        }
    }
    CHECK(to_status(sell_plan(p->st, p->ar, n, p->rowptr, p->sell_off, p->sell_perm, sell_budget(nnz),
                              &p->sell_ok, &p->sell_sorted, &p->sell_total, &p->sell_wuni),
                    "sliced ELL"));
    if (p->need_adjoint)
        CHECK(to_status(sell_plan(p->st, p->ar, n, p->trp, p->tsell_off, p->tsell_perm, sell_budget(nnz),
                                  &p->tsell_ok, &p->tsell_sorted, &p->tsell_total, &p->tsell_wuni),
                        "sliced ELL (A^T)"));
    if (p->ar.short_) return short_of(est.total());

    // The exact size, now that the counts are known.
    const Layout ex = layout_of(p, true);
    if (ex.total() > workspace_bytes) return short_of(ex.total());
    carve_phase2(p, p->ar);
    if (p->ar.short_ || p->ar.lo - lo1 != ex.p2) return short_of(ex.total());

    // Sliced-ELL patterns (dropped when a column offset does not fit 16 bits).
    if (p->sell_ok) {
        bool ok = false;
        CHECK(to_status(sell_fill_pattern(p->st, n, p->rowptr, p->colind, p->sell_off,
                                          p->sell_sorted ? p->sell_perm : nullptr, p->sell_col,
                                          p->sell_src, p->d_flags, &ok), "sliced ELL"));
        if (!ok) p->sell_ok = false;
    }
    if (p->tsell_ok) {
        bool ok = false;
        CHECK(to_status(sell_fill_pattern(p->st, n, p->trp, p->tci, p->tsell_off,
                                          p->tsell_sorted ? p->tsell_perm : nullptr, p->tsell_col,
                                          p->tsell_src, p->d_flags, &ok), "sliced ELL (A^T)"));
        if (!ok) p->tsell_ok = false;
    }
    if (!p->sell_ok) {
        p->sell_col = nullptr;
        p->sell_src = nullptr;
        p->sell_total = 0;
        p->sell_wuni = 0;
    }
    if (!p->sell_sorted) p->sell_perm = nullptr;
    if (!p->tsell_ok) {
        p->tsell_col = nullptr;
        p->tsell_src = nullptr;
        p->tsell_total = 0;
        p->tsell_wuni = 0;
    }
    if (!p->tsell_sorted) p->tsell_perm = nullptr;
    p->sell_wmax = max_row_len(p->st, n, p->rowptr, p->d_flags);
    if (p->need_adjoint) p->tsell_wmax = max_row_len(p->st, n, p->trp, p->d_flags);
    CHECK(refresh_values(p));

    if (p->o.spmv_lanes == kSell && !p->sell_col)
        return fail(GMRES_EINVAL, "spmv_lanes = -64 needs a sliced-ELL copy (column offsets col - row "
                                  "within +-32767, padding within budget)");
    p->L = p->o.spmv_lanes != 0 ? p->o.spmv_lanes
                                : default_lanes(n, nnz, p->sell_col != nullptr, p->sell_total);
    if (nsys == 1) {
        CHECK(build_slots(p));
        CHECK(init_krylov(p));
        if (!(p->block = gm::block_new())) return fail(GMRES_EINVAL, "host allocation of the plan failed");
    }
    if (p->bV) CHECK(init_batched(p));
    p->batch_wg = p->o.batch_wg > 0 ? p->o.batch_wg : 256;
    p->batch_L = p->o.batch_lanes > 0 ? p->o.batch_lanes : 8;
    HIP_OK(hipStreamSynchronize(p->st));
    CHECK(leave(p));
    return GMRES_OK;
}

size_t gmres_workspace_bytes(int32_t nsys, const int64_t* sys_row_off_h, const int64_t* sys_zcol_off_h,
                             int64_t nnz, int64_t z_nnz, const gmres_opts* opts, int32_t need_adjoint) {
    gmres_plan_s* p = new (std::nothrow) gmres_plan_s();
    if (!p) return 0;
    size_t bytes = 0;
    if (check_args(p, nsys, sys_row_off_h, sys_zcol_off_h, nullptr, nullptr, nullptr, nnz, nullptr,
                   nullptr, nullptr, z_nnz, opts, need_adjoint, false) == GMRES_OK)
        bytes = layout_of(p, false).total();
    delete p;
    return bytes;
}

size_t gmres_workspace_required(void) { return g_ws_required; }

gmres_status gmres_setup(gmres_plan* out, int32_t nsys, const int64_t* sys_row_off_h,
                         const int64_t* sys_zcol_off_h, const int32_t* rowptr,
                         const int32_t* colind, const double* vals, int64_t nnz,
                         const int32_t* z_rowptr, const int32_t* z_colind, const double* z_vals,
                         int64_t z_nnz, const gmres_opts* opts, int32_t need_adjoint,
                         void* workspace, size_t workspace_bytes, hipStream_t stream) {
    TraceRange tr_("gmres_setup");
    if (!out) return fail(GMRES_EINVAL, "out is NULL");
    *out = nullptr;
    g_ws_required = 0;
    gmres_plan_s* p = new (std::nothrow) gmres_plan_s();
    if (!p) return fail(GMRES_EINVAL, "host allocation of the plan failed");
    gmres_status s = setup_impl(p, nsys, sys_row_off_h, sys_zcol_off_h, rowptr, colind, vals, nnz,
                                z_rowptr, z_colind, z_vals, z_nnz, opts, need_adjoint, workspace,
                                workspace_bytes, stream);
    if (s != GMRES_OK) {
        std::string msg = g_last_error;
        gmres_destroy(p);
        g_last_error = msg;
        return s;
    }
    *out = p;
    return GMRES_OK;
}

gmres_status gmres_set_stream(gmres_plan p, hipStream_t stream) {
    if (!p) return fail(GMRES_EINVAL, "plan is NULL");
    p->user_stream = stream;
    return GMRES_OK;
}

gmres_status gmres_solve(gmres_plan p, const double* b, const double* x0, double* x,
                         gmres_info* info_h) {
    TraceRange tr_("gmres_solve");
    if (!p || !b || !x) return fail(GMRES_EINVAL, "plan, b and x are required");
    if (p->nsys != 1) return fail(GMRES_EINVAL, "gmres_solve needs a single-system plan");
    if (x == b) return fail(GMRES_EINVAL, "x must not alias b");
    const auto t0 = std::chrono::steady_clock::now();
    CHECK(enter(p));
    gmres_info info{};
    p->hist_pos = 0;
    p->timer.reset();
    if (p->o.precision == GMRES_FP64) {
        CHECK(solve_f64(p, 0, b, x0, x, p->o.rtol, p->o.r0_norm_override, p->o.max_iters, &info));
    } else {
        CHECK(solve_mixed(p, b, x0, x, &info));
    }
    p->hist_len = std::min<int64_t>(info.iters, p->hist_cap);
    double nrm = 0;
    CHECK(true_residual(p, b, x, &nrm));
    info.rel_res_true = info.rho0 > 0 ? nrm / info.rho0 : 0.0;
    CHECK(leave(p));
    info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_h) *info_h = info;
    if (info.status == kStatusNonFinite) return fail(GMRES_ENONFINITE, "non-finite value in b, x0 or the iteration");
    return (gmres_status)info.status;
}

static gmres_status solve_block_impl(gmres_plan p, int32_t k, int32_t m_block, const double* B,
                                     const double* X0, double* X, void* work, size_t work_bytes,
                                     gmres_info* info_h) {
    TraceRange tr_("gmres_solve_block");
    if (!p || !B || !X) return fail(GMRES_EINVAL, "plan, B and X are required");
    if (p->nsys != 1) return fail(GMRES_EINVAL, "gmres_solve_block needs a single-system plan");
    if (p->o.adapt_rmax > 0) return fail(GMRES_EINVAL, "gmres_solve_block does not run adaptive deflation");
    if (p->R > gm::kBlockZMax)
        return fail(GMRES_EINVAL, "gmres_solve_block supports deflation bases of at most 64 columns");
    if (k < 1 || k > 16) return fail(GMRES_EINVAL, "k must be in [1, 16]");
    if (m_block < 1 || m_block > gm::kBlockStepsMax) return fail(GMRES_EINVAL, "m_block must be in [1, 16]");
    if (X == B) return fail(GMRES_EINVAL, "X must not alias B");
    const size_t need = gm::block_workspace_bytes(p->n, m_block);
    if (!work || work_bytes < need) {
        g_ws_required = need;
        return fail(GMRES_EWORKSPACE, "block workspace too small: " + std::to_string(need) + " bytes needed");
    }
    if (reinterpret_cast<uintptr_t>(work) & 255) return fail(GMRES_EINVAL, "block workspace must be 256-byte aligned");
    const auto t0 = std::chrono::steady_clock::now();
    CHECK(enter(p));
    CHECK(to_status(gm::block_bind(p->block, work, work_bytes, p->st, p->n, m_block), "block workspace"));
    // Timing (set_timing > 0): every block kernel launch carries its events.
    struct Hook final : gm::BlockTimer {
        gmres_plan_s* p;
        int cur = -1;            // block step of the launches being recorded (-1: outside steps)
        size_t cyc_first = 0;    // first record of the current cycle
        explicit Hook(gmres_plan_s* q) : p(q) {}
        void begin(int kind, double bytes) override {
            Timer& t = p->timer;
            const int e0 = t.used++;
            t.used++;
            arm_kernel_events(t.ev(e0), t.ev(e0 + 1));
            t.recs.push_back({kind, 0, cur, bytes, e0});
        }
        void end() override {
            if (disarm_kernel_events()) p->timer.recs.back().cycle = -1;
        }
        void step(int j) override { cur = j; }
        void cycle_done(int jd) override {
            auto& recs = p->timer.recs;
            for (size_t i = cyc_first; i < recs.size(); ++i)
                if (recs[i].j >= jd) recs[i].cycle = -1;
            cyc_first = recs.size();
            cur = -1;
        }
    } hook(p);
    p->timer.reset();
    gm::BlockArgs a{p->st, p->rowptr, p->colind, p->vals, k, m_block, p->o.rtol, p->o.max_iters, B, X0, X,
                    p->nnz, p->timer.period > 0 ? &hook : nullptr, p->R, p->ztrp, p->ztci, p->ztv, p->zrp,
                    p->zci, p->zv, p->azrp, p->azci, p->azv, p->Einv};
    gm::BlockResult r;
    const int s = gm::block_solve(p->block, a, &r);
    if (p->timer.period > 0) {
        Timer& t = p->timer;
        for (const auto& rec : t.recs) {
            if (rec.cycle < 0) continue;
            float ms = 0.f;
            hipEventElapsedTime(&ms, t.pool[rec.ev], t.pool[rec.ev + 1]);
            t.launches[rec.kind] += 1;
            t.ms[rec.kind] += ms;
            t.bytes[rec.kind] += rec.bytes;
        }
        t.recs.clear();
        t.used = 0;
    }
    if (s == kStatusInval) {
        leave(p);
        return fail(GMRES_EINVAL, "a column of B - A X0 is zero (or not finite)");
    }
    CHECK(to_status(s, "block GMRES"));
    CHECK(leave(p));
    gmres_info info{};
    info.status = r.status;
    info.iters = r.steps;
    info.cycles = r.cycles;
    info.rho0 = r.rho0;
    info.rel_res = r.rel_res_est;
    info.rel_res_true = r.rel_res_true;
    info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_h) *info_h = info;
    return (gmres_status)info.status;
}

size_t gmres_block_workspace_bytes(gmres_plan p, int32_t m_block) {
    if (!p || m_block < 1 || m_block > gm::kBlockStepsMax) return 0;
    return gm::block_workspace_bytes(p->n, m_block);
}

gmres_status gmres_solve_block(gmres_plan p, int32_t k, int32_t m_block, const double* B,
                               const double* X0, double* X, void* work, size_t work_bytes,
                               gmres_info* info_h) {
    return solve_block_impl(p, k, m_block, B, X0, X, work, work_bytes, info_h);
}

gmres_status gmres_solve_block_noalloc(gmres_plan p, int32_t k, int32_t m_block, const double* B,
                                       const double* X0, double* X, gmres_info* info_h) {
    if (!p) return fail(GMRES_EINVAL, "plan is NULL");
    if (m_block < 1 || m_block > gm::kBlockStepsMax) return fail(GMRES_EINVAL, "m_block must be in [1, 16]");
    size_t cap = 0;
    void* work = gm::static_scratch(p->device, &cap);
    if (!work) return fail(GMRES_EDEVICE, "the static scratch address is unavailable on this device");
    const size_t need = gm::block_workspace_bytes(p->n, m_block);
    if (need > cap)
        return fail(GMRES_EINVAL, "block solve needs " + std::to_string(need) +
                                      " bytes of scratch; the static scratch holds " + std::to_string(cap));
    return solve_block_impl(p, k, m_block, B, X0, X, work, cap, info_h);
}

gmres_status gmres_adjoint(gmres_plan p, const double* x, const double* grad_x, double* grad_b,
                           double* grad_vals, gmres_info* info_h) {
    TraceRange tr_("gmres_adjoint");
    if (!p || !x || !grad_x) return fail(GMRES_EINVAL, "plan, x and grad_x are required");
    if (!p->need_adjoint) return fail(GMRES_EINVAL, "plan was built without need_adjoint");
    const auto t0 = std::chrono::steady_clock::now();
    CHECK(enter(p));
    gmres_info info{};
    p->hist_pos = 0;
    p->timer.reset();
    CHECK(solve_f64(p, 1, grad_x, nullptr, p->dvec, p->o.rtol, 0.0, p->o.max_iters, &info));
    if (grad_b) launch_copy(p->st, p->dvec, grad_b, p->n);
    if (grad_vals)
        gm::grad_vals(p->st, p->n, p->rowptr, p->colind, p->dvec, x, grad_vals);
    // True residual of the adjoint system ||grad_x - A^T lambda||.
    const int slot = p->o.m + 1;
    launch_residual_f64(p->st, p->L, p->NB, (int)p->n, p->trp, p->tci, p->tv, p->dvec, grad_x, p->w,
                        p->part, slot);
    launch_sum_slot(p->st, p->part, p->NB, slot, p->scal);
    double h = 0;
    HIP_OK(hipMemcpyAsync(&h, p->scal, sizeof(double), hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    info.rel_res_true = info.rho0 > 0 ? std::sqrt(h) / info.rho0 : 0.0;
    CHECK(leave(p));
    info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info_h) *info_h = info;
    return (gmres_status)info.status;
}

gmres_status gmres_update_values(gmres_plan p, const double* vals) {
    TraceRange tr_("gmres_update_values");
    if (!p || (!vals && p->nnz > 0)) return fail(GMRES_EINVAL, "plan and vals are required");
    CHECK(enter(p));
    if (p->nnz > 0)
        HIP_OK(hipMemcpyAsync(p->vals, vals, p->nnz * sizeof(double), hipMemcpyDeviceToDevice, p->st));
    SetupArgs sa{p->st, p->nsys, p->n, p->nnz, p->znnz, p->R, p->d_row_off, p->d_zcol_off,
                 p->rowptr, p->colind, p->vals, p->zrp, p->zci, p->zv};
    CHECK(to_status(setup_validate(sa, p->d_flags), "value validation"));
    CHECK(refresh_values(p));
    if (p->ncont > 0) {
        // Attached continuation plans hold the old values: detach them all.
        std::fill(p->cont.begin(), p->cont.end(), nullptr);
        std::fill(p->cont_steps.begin(), p->cont_steps.end(), 0);
        p->ncont = 0;
        HIP_OK(hipMemsetAsync(p->d_hand, 0, p->nsys * sizeof(int64_t), p->st));
    }
    CHECK(leave(p));
    return GMRES_OK;
}

gmres_status gmres_spmv(gmres_plan p, const double* x, double* y) {
    if (!p || !x || !y) return fail(GMRES_EINVAL, "plan, x and y are required");
    CHECK(enter(p));
    spmv_f64(p, p->L, p->NB > 0 ? p->NB : 1, x, y);
    HIP_OK(hipGetLastError());
    CHECK(leave(p));
    HIP_OK(hipStreamSynchronize(p->st));
    return GMRES_OK;
}

int64_t gmres_history(gmres_plan p, double* hist_h, int64_t cap) {
    if (!p || !hist_h || !p->hist) return -1;
    const int64_t k = std::min<int64_t>(std::min<int64_t>(cap, p->hist_len), p->hist_cap);
    if (k > 0 && hipMemcpy(hist_h, p->hist, k * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    return k;
}

static void drop_graphs(gmres_plan_s* p) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            if (p->gexec[a][b]) hipGraphExecDestroy(p->gexec[a][b]);
            if (p->graph[a][b]) hipGraphDestroy(p->graph[a][b]);
            p->gexec[a][b] = nullptr;
            p->graph[a][b] = nullptr;
        }
}

static gmres_status init_batched(gmres_plan_s* p) {
    const int ns = p->nsys;
    const int m = p->o.m;
    // Largest systems first: order by nnz, then rows.
    std::vector<int32_t> rp_at(ns + 1);
    for (int s = 0; s <= ns; ++s)
        HIP_OK(hipMemcpy(&rp_at[s], p->rowptr + p->row_off[s], sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int> order(ns);
    for (int s = 0; s < ns; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int64_t wa = (int64_t)(rp_at[a + 1] - rp_at[a]) + (p->row_off[a + 1] - p->row_off[a]);
        const int64_t wb = (int64_t)(rp_at[b + 1] - rp_at[b]) + (p->row_off[b + 1] - p->row_off[b]);
        return wa > wb;
    });
    std::vector<int64_t> voff(ns), woff(ns);
    int64_t acc = 0;
    for (int s = 0; s < ns; ++s) {
        const int64_t ld = (p->row_off[s + 1] - p->row_off[s] + 1) & ~int64_t(1);
        voff[s] = (int64_t)(m + 1) * acc;
        woff[s] = 3 * acc;
        acc += ld;
    }
    HIP_OK(hipMemcpy(p->border, order.data(), ns * sizeof(int), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->d_v_off, voff.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->d_w_off, woff.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice));
    // Padding rows of the work vectors (and, for batches, of the basis) read as zero.
    HIP_OK(hipMemsetAsync(p->bW, 0, 3 * (size_t)(p->n + ns) * sizeof(double), p->st));
    if (ns > 1) {
        HIP_OK(hipMemsetAsync(p->d_hand, 0, ns * sizeof(int64_t), p->st));
        p->cont.assign(ns, nullptr);
        p->cont_steps.assign(ns, 0);
        HIP_OK(hipMemsetAsync(p->bV, 0, (size_t)(m + 1) * (p->n + ns) * sizeof(double), p->st));
        if (p->R > 0) {
            HIP_OK(hipMemsetAsync(p->azc1, 0xFF, 2 * (size_t)p->n * sizeof(int), p->st));
            refresh_ell1(p);
        }
    }
    return GMRES_OK;
}

static gmres_status run_batched(gmres_plan_s* p, const double* b, const double* x0, double* x,
                                int64_t max_iters, int wg, int lanes) {
    HIP_OK(hipMemsetAsync(p->bticket, 0, sizeof(int), p->st));
    // A single-system plan lends its Krylov basis: clear it so that the padding
    // row of the batched layout reads as zero.
    if (p->nsys == 1)
        HIP_OK(hipMemsetAsync(p->bV, 0, (size_t)(p->o.m + 1) * (p->n + 1) * sizeof(double), p->st));
    BatchArgs a{};
    a.st = p->st;
    a.nsys = p->nsys;
    a.m = p->o.m;
    a.L = lanes;
    a.wg = wg;
    a.max_iters = max_iters;
    a.rtol = p->o.rtol;
    a.row_off = p->d_row_off;
    a.zcol_off = p->d_zcol_off;
    a.e_off = p->d_e_off;
    a.v_off = p->d_v_off;
    a.w_off = p->d_w_off;
    a.zc1 = p->zc1;
    a.zv1 = p->zv1;
    a.az2c = p->azc1;
    a.az2v = p->azv1;
    if (p->sell_col && !p->sell_perm) {     // rows in order: a system's rows are a range of positions
        a.sell_off = p->sell_off;
        a.sell_wuni = p->sell_wuni;
        a.sell_col = p->sell_col;
        a.sell_val = p->sell_v64;
    }
    a.order = p->border;
    a.hand = p->ncont > 0 ? p->d_hand : nullptr;
    a.rec = p->ncont > 0 ? p->hrec_d : nullptr;
    if (a.rec) std::memset(p->hrec_h, 0, (size_t)p->nsys * sizeof(HandRec));   // the last launch has ended
    a.rowptr = p->rowptr;
    a.colind = p->colind;
    a.vals = p->vals;
    a.azrp = p->azrp;
    a.azci = p->azci;
    a.azv = p->azv;
    a.zrp = p->zrp;
    a.zci = p->zci;
    a.zv = p->zv;
    a.ztrp = p->ztrp;
    a.ztci = p->ztci;
    a.ztv = p->ztv;
    a.Einv = p->Einv;
    a.b = b;
    a.x0 = x0;
    a.x = x;
    a.V = p->bV;
    a.W = p->bW;
    a.ticket = p->bticket;
    a.out_i = p->bout_i;
    a.out_d = p->bout_d;
    int cus = 0;
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
    const int per_cu = std::max(1, 1024 / wg);
    const int nwg = std::max(1, std::min(p->nsys, cus * per_cu));
    launch_batched(a, nwg);
    HIP_OK(hipGetLastError());
    return GMRES_OK;
}

gmres_status gmres_batched_attach(gmres_plan p, int32_t s, gmres_plan sub, int64_t steps) {
    if (!p || p->nsys < 2 || !p->d_hand) return fail(GMRES_EINVAL, "attach needs a plan of several systems");
    if (s < 0 || s >= p->nsys) return fail(GMRES_EINVAL, "system index out of range");
    if (sub) {
        const int64_t rows = p->row_off[s + 1] - p->row_off[s];
        const int64_t r_s = p->zcol_off[s + 1] - p->zcol_off[s];
        if (sub == p || sub->nsys != 1 || sub->n != rows || sub->R != r_s)
            return fail(GMRES_EINVAL, "the attached plan must be a single-system plan of system s's size and r");
        if (sub->o.m != p->o.m || sub->o.adapt_rmax > 0 || sub->device != p->device)
            return fail(GMRES_EINVAL, "the attached plan must share m and the device, without adaptive deflation");
        if (steps < 1) return fail(GMRES_EINVAL, "steps must be >= 1");
        for (int t = 0; t < p->nsys; ++t)
            if (t != s && p->cont[t] == sub)
                return fail(GMRES_EINVAL, "a plan continues at most one system of the batch");
    }
    HIP_OK(hipSetDevice(p->device));
    if (sub && !p->hrec_h) {
        HIP_OK(hipHostMalloc((void**)&p->hrec_h, (size_t)p->nsys * sizeof(HandRec),
                             hipHostMallocCoherent | hipHostMallocMapped));
        HIP_OK(hipHostGetDevicePointer((void**)&p->hrec_d, p->hrec_h, 0));
    }
    if (!p->cont[s] && sub) ++p->ncont;
    if (p->cont[s] && !sub) --p->ncont;
    p->cont[s] = sub;
    p->cont_steps[s] = sub ? steps : 0;
    HIP_OK(hipMemcpyAsync(p->d_hand + s, &p->cont_steps[s], sizeof(int64_t), hipMemcpyHostToDevice, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    return GMRES_OK;
}

namespace {

// System s of a batched solve, continued on its attached plan q: restarted
// GMRES carries only the iterate from one cycle to the next, so restarting
// from the batch's x_s (with the batch's rho0 as the tolerance reference) is
// the same iteration (Sec. 3.2, restarts); P r is unchanged by the coarse
// correction the batched kernel applied to x_s, since P A Z = 0.
struct Continuation {
    gmres_plan_s* q = nullptr;
    int s = 0;
    int stage = 0;   // 0 not started, 1 cycles in flight, 2 final copy in flight, 3 done
    int slot = 0;
    int saved_period = 0;
    std::unique_ptr<EngineRun> run;
    std::chrono::steady_clock::time_point t0;
    double ms = 0;
    Ctrl out{};
};

gmres_status cont_start(gmres_plan_s* p, Continuation& c, const double* b, double* x, double rho0,
                        int64_t steps_left) {
    gmres_plan_s* q = c.q;
    const int64_t off = p->row_off[c.s];
    // x_s is in memory (the launch released it before the flag, or has
    // ended), and these kernels start after this point.
    launch_copy(q->st, b + off, q->bws, q->n);
    launch_copy(q->st, x + off, q->xh, q->n);
    c.saved_period = q->timer.period;
    q->timer.period = 0;   // kernel timing is not collected for continuations
    q->hist_pos = 0;
    c.run.reset(new EngineRun(q, 0, kPrecF64));
    CHECK(engine_start(*c.run, q->bws, p->o.rtol, rho0, steps_left, false));
    c.stage = 1;
    return GMRES_OK;
}

// Advances one continuation without blocking; *moved reports progress.
gmres_status cont_poll(gmres_plan_s* p, Continuation& c, double* x, bool* moved) {
    gmres_plan_s* q = c.q;
    *moved = false;
    if (c.stage == 1) {
        bool ready = false;
        CHECK(engine_step(*c.run, false, &ready));
        if (!ready) return GMRES_OK;
        *moved = true;
        if (c.run->exhausted) return fail(GMRES_EDEVICE, "continuation loop did not terminate");
        if (!c.run->finished) return GMRES_OK;
        // x_s = x_hat + Z E^{-1} Z^T r, then the final control block; the copy
        // lands after the last enqueued cycle's snapshot in the same slot.
        launch_correct(q->st, q->NB, (int)q->n, q->zrp, q->zci, q->zv, q->s_res, q->R, q->xh,
                       x + p->row_off[c.s]);
        c.slot = (int)(c.run->c & 1);
        HIP_OK(hipMemcpyAsync(&q->ctrl_h[c.slot], q->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, q->st));
        HIP_OK(hipEventRecord(q->ev_cyc[c.slot], q->st));
        c.stage = 2;
        return GMRES_OK;
    }
    if (c.stage == 2) {
        const hipError_t e = hipEventQuery(q->ev_cyc[c.slot]);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            return GMRES_OK;
        }
        HIP_OK(e);
        c.run->span[0].stop();
        c.run->span[1].stop();
        c.out = q->ctrl_h[c.slot];
        q->timer.period = c.saved_period;
        q->hist_len = std::min<int64_t>(c.out.its, q->hist_cap);
        c.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c.t0).count();
        c.stage = 3;
        *moved = true;
    }
    return GMRES_OK;
}

// Runs the continuations of the systems that leave the batched launch, at
// most kActive at a time (each on its plan's own stream), polling from this
// thread: a system starts as soon as its host-visible record is flagged,
// while the launch still runs; once the launch has ended, one more scan
// finds every remaining one.
gmres_status run_continuations(gmres_plan_s* p, std::vector<Continuation>& cs, const double* b, double* x) {
    constexpr int kActive = 16;
    TraceRange tr_("batched continuations");
    const int ns = p->nsys;
    HIP_OK(hipEventRecord(p->ev_out, p->st));   // the batched launch has ended
    std::vector<int> watch;
    for (int s = 0; s < ns; ++s)
        if (p->cont[s]) watch.push_back(s);
    std::vector<int64_t> its0;
    std::vector<double> rho0;
    bool launch_done = false, scanned_after = false;
    size_t next = 0, done = 0;
    int active = 0;
    for (;;) {
        if (!launch_done) {
            const hipError_t e = hipEventQuery(p->ev_out);
            if (e == hipSuccess) launch_done = true;
            else if (e == hipErrorNotReady) (void)hipGetLastError();
            else HIP_OK(e);
        }
        const bool final_scan = launch_done && !scanned_after;
        for (size_t k = 0; k < watch.size(); ++k) {
            const int s = watch[k];
            if (s < 0 || __atomic_load_n(&p->hrec_h[s].flag, __ATOMIC_ACQUIRE) == 0) continue;
            cs.emplace_back();
            cs.back().q = p->cont[s];
            cs.back().s = s;
            cs.back().t0 = std::chrono::steady_clock::now();   // waiting for a slot counts too
            its0.push_back(p->hrec_h[s].its);
            rho0.push_back(p->hrec_h[s].rho0);
            watch[k] = -1;
        }
        if (final_scan) scanned_after = true;
        while (active < kActive && next < cs.size()) {
            Continuation& c = cs[next];
            CHECK(cont_start(p, c, b, x, rho0[next], p->o.max_iters - its0[next]));
            ++next;
            ++active;
        }
        bool any = false;
        for (size_t i = 0; i < next; ++i) {
            Continuation& c = cs[i];
            if (c.stage == 0 || c.stage == 3) continue;
            bool moved = false;
            CHECK(cont_poll(p, c, x, &moved));
            any = any || moved;
            if (c.stage == 3) {
                --active;
                ++done;
            }
        }
        if (scanned_after && done == cs.size()) break;
        if (!any) std::this_thread::yield();
    }
    return GMRES_OK;
}

}  // namespace

gmres_status gmres_solve_batched(gmres_plan p, const double* b, const double* x0, double* x,
                                 gmres_info* infos_h) {
    TraceRange tr_("gmres_solve_batched");
    if (!p || !b || !x) return fail(GMRES_EINVAL, "plan, b and x are required");
    if (p->o.m > 64) return fail(GMRES_EINVAL, "the batched solver supports m <= 64");
    if (x == b) return fail(GMRES_EINVAL, "x must not alias b");
    if (!p->bV) return fail(GMRES_EINVAL, "the batched solver supports m <= 64");
    const auto t0 = std::chrono::steady_clock::now();
    CHECK(enter(p));
    CHECK(run_batched(p, b, x0, x, p->o.max_iters, p->batch_wg, p->batch_L));
    const int ns = p->nsys;
    double* nr = p->bout_d + 4 * (int64_t)ns;
    std::vector<int64_t> oi(3 * (size_t)ns);
    std::vector<double> od(5 * (size_t)ns);
    // Systems that reach their step limit go on on their attached plans.
    std::vector<Continuation> cs;
    if (p->ncont > 0) {
        cs.reserve(p->ncont);
        CHECK(run_continuations(p, cs, b, x));
    }
    launch_seg_resid(p->st, ns, p->d_row_off, p->rowptr, p->colind, p->vals, x, b, nr);
    if (ns == 1) p->last_prec = -1;   // the shared basis (and its padding) is cleared before the next solve
    HIP_OK(hipMemcpyAsync(oi.data(), p->bout_i, oi.size() * sizeof(int64_t), hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipMemcpyAsync(od.data(), p->bout_d, od.size() * sizeof(double), hipMemcpyDeviceToHost, p->st));
    HIP_OK(hipStreamSynchronize(p->st));
    CHECK(leave(p));
    int clk_khz = 0;
    HIP_OK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, p->device));
    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::vector<const Continuation*> by_sys(ns, nullptr);
    for (const Continuation& c : cs) by_sys[c.s] = &c;
    gmres_status worst = GMRES_OK;
    for (int s = 0; s < ns; ++s) {
        gmres_info in{};
        in.iters = oi[3 * s];
        in.cycles = (int32_t)oi[3 * s + 1];
        in.status = (int32_t)oi[3 * s + 2];
        in.rho0 = od[4 * s];
        in.rel_res = od[4 * s + 1];
        in.rel_res_true = in.rho0 > 0 ? std::sqrt(od[4 * ns + s]) / in.rho0 : 0.0;
        in.solve_ms = clk_khz > 0 ? (od[4 * s + 3] - od[4 * s + 2]) / (double)clk_khz : wall;
        if (in.status == kStatusHandoff && !by_sys[s])
            return fail(GMRES_EDEVICE, "a system left the batch without being continued");
        if (const Continuation* c = by_sys[s]) {
            in.iters += c->out.its;
            in.cycles += c->out.cycles;
            in.status = c->out.status;
            in.rel_res = in.rho0 > 0 ? c->out.beta / in.rho0 : 0.0;
            in.solve_ms += c->ms;
        }
        if (infos_h) infos_h[s] = in;
        if (worst == GMRES_OK && in.status != GMRES_OK) worst = (gmres_status)in.status;
    }
    if (worst < 0) return fail(worst, "a system of the batch failed");
    return worst;
}

// Autotune cache (GMRES_TUNE_CACHE names a text file): one line per tuned
// plan shape, "<key>\t<lanes> <grid> <batch workgroup> <batch lanes>"; the
// key holds the device (architecture, compute units) and everything the
// choices depend on.  The last line with a matching key wins; a choice the
// plan cannot run (sliced ELL not built, grid above the resident cap) is
// ignored and the plan is tuned again.  Appends are not locked against other
// processes writing the same file.
static std::string tune_key(const gmres_plan_s* p) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return std::string();
    std::ostringstream k;
    k << "v1 arch=" << prop.gcnArchName << " cu=" << prop.multiProcessorCount << " nsys=" << p->nsys
      << " n=" << p->n << " nnz=" << p->nnz << " R=" << p->R << " m=" << p->o.m
      << " prec=" << p->o.precision << " ortho=" << p->o.ortho << " sell=" << (p->sell_col ? p->sell_total : -1);
    return k.str();
}

static bool tune_cache_read(const char* path, const std::string& key, int32_t (&v)[4]) {
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        std::istringstream vs(line.substr(tab + 1));
        int32_t t[4];
        if (vs >> t[0] >> t[1] >> t[2] >> t[3]) {
            for (int i = 0; i < 4; ++i) v[i] = t[i];
            found = true;
        }
    }
    return found;
}

static void tune_cache_append(const char* path, const std::string& key, const gmres_plan_s* p) {
    std::ofstream out(path, std::ios::app);
    if (out) out << key << '\t' << p->L << ' ' << p->NB << ' ' << p->batch_wg << ' ' << p->batch_L << '\n';
}

static bool tune_choice_valid(const gmres_plan_s* p, const int32_t (&v)[4]) {
    const bool lanes_ok = (v[0] == kSell && p->sell_col) ||
                          (v[0] == -256 || v[0] == 2 || v[0] == 4 || v[0] == 8 || v[0] == 16 || v[0] == 32);
    const bool nb_ok = v[1] >= 1 && v[1] <= p->NB_cap;
    const bool batch_ok = (v[2] == 256 || v[2] == 512 || v[2] == 1024) &&
                          (v[3] == 4 || v[3] == 8 || v[3] == 16 || v[3] == 32);
    return lanes_ok && nb_ok && batch_ok;
}

gmres_status gmres_autotune(gmres_plan p, int32_t* chosen_h) {
    TraceRange tr_("gmres_autotune");
    if (!p) return fail(GMRES_EINVAL, "plan is NULL");
    const char* cache = std::getenv("GMRES_TUNE_CACHE");
    const std::string key = (cache && cache[0]) ? tune_key(p) : std::string();
    int32_t cached[4];
    if (!key.empty() && tune_cache_read(cache, key, cached) && tune_choice_valid(p, cached)) {
        p->L = cached[0];
        p->NB = cached[1];
        p->batch_wg = cached[2];
        p->batch_L = cached[3];
        drop_graphs(p);
        if (chosen_h)
            for (int i = 0; i < 4; ++i) chosen_h[i] = cached[i];
        return GMRES_OK;
    }
    CHECK(enter(p));
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    auto time_it = [&](auto&& fn, int reps) -> double {
        fn();
        hipEventRecord(e0, p->st);
        for (int r = 0; r < reps; ++r) fn();
        hipEventRecord(e1, p->st);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        return ms / reps;
    };
    if (p->nsys == 1) {
        // SpMV lanes per row, then the streaming grid size (SpMV + a mid-cycle
        // pass 2, the dominant Arnoldi kernel).
        const int n = (int)p->n;
        launch_fill(p->st, (double*)p->V, (int64_t)(p->o.m + 1) * p->ldv, 1.0 / std::sqrt((double)n));
        launch_fill(p->st, p->w, n, 1.0);
        launch_fill(p->st, p->coef1, p->o.m + 1, 1e-3);
        double best = 1e30;
        int bestL = p->L;
        for (int L : {kSell, -256, 2, 4, 8, 16, 32}) {
            if (L == kSell && !p->sell_col) continue;
            const double t = time_it([&] { spmv_f64(p, L, p->NB, (double*)p->V, p->y); }, 10);
            if (t < best) { best = t; bestL = L; }
        }
        p->L = bestL;
        const int nb_cap = p->NB_cap;
        double bestt = 1e30;
        int bestNB = p->NB;
        const int nv = std::max(1, p->o.m / 2);
        for (int nb : {256, 512, 768, 1024, 1536, 2048}) {
            if (nb > nb_cap) continue;
            const int saved = p->NB;
            p->NB = nb;
            const int tprec = p->o.precision == GMRES_MIXED_F16 ? kPrecF16
                              : (p->o.precision == GMRES_MIXED_F32 ? kPrecF32 : kPrecF64);
            EngineArgs a = make_args(p, 0, tprec);
            const double t = time_it([&] {
                spmv_f64(p, p->L, nb, (double*)p->V, p->y);
                launch_pass_probe(a, 1, nv);
                launch_pass_probe(a, 2, nv);
                launch_pass_probe(a, 3, nv);
            }, 6);
            p->NB = saved;
            if (t < bestt) { bestt = t; bestNB = nb; }
        }
        p->NB = bestNB;
        CHECK(clear_typed(p));
        p->last_prec = kPrecF64;
        drop_graphs(p);
    } else {
        // Batched: workgroup size and SpMV lanes, timed on one restart cycle.
        double* xx = p->btune_x;
        double* ones = p->btune_b;
        launch_fill(p->st, ones, p->n, 1.0);
        double best = 1e30;
        for (int wg : {256, 512}) {
            for (int L : {4, 8, 16}) {
                const double t = time_it([&] {
                    run_batched(p, ones, nullptr, xx, p->o.m, wg, L);
                }, 2);
                if (t < best) { best = t; p->batch_wg = wg; p->batch_L = L; }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    HIP_OK(hipStreamSynchronize(p->st));
    CHECK(leave(p));
    if (!key.empty()) tune_cache_append(cache, key, p);
    if (chosen_h) {
        chosen_h[0] = p->L;
        chosen_h[1] = p->NB;
        chosen_h[2] = p->batch_wg;
        chosen_h[3] = p->batch_L;
    }
    return GMRES_OK;
}

gmres_status gmres_set_timing(gmres_plan p, int32_t period) {
    if (!p) return fail(GMRES_EINVAL, "plan is NULL");
    if (period < 0) return fail(GMRES_EINVAL, "timing period must be >= 0");
    p->timer.period = period;
    p->timer.reset();
    return GMRES_OK;
}

gmres_status gmres_kernel_times(gmres_plan p, double* out_h) {
    if (!p || !out_h) return fail(GMRES_EINVAL, "plan and out_h are required");
    for (int k = 0; k < Timer::kKinds; ++k) {
        out_h[3 * k + 0] = p->timer.launches[k];
        out_h[3 * k + 1] = p->timer.ms[k];
        out_h[3 * k + 2] = p->timer.bytes[k];
    }
    return GMRES_OK;
}

}  // extern "C"
