// Device kernels of one deflated GMRES(m) restart cycle on a single system.
//
// Arithmetic follows arXiv 1906.04051, Sec. 3.2-3.3: Arnoldi (eq. krylov-basis)
// with classical Gram-Schmidt applied twice (CGS2 -- the paper uses modified
// Gram-Schmidt; both build the same orthonormal basis in exact arithmetic),
// plane rotations of the Hessenberg matrix and the residual estimate
// |gamma_{k+1}| (eqs. arg, hessenberg, res), x_m = x_0 + V_m y_m (eq. new_sol),
// restarts from x_m (GMRES(m)) and the relative-residual test (eq. relative).
// The operator is P A with P = I - A Z E^{-1} Z^T, E = Z^T A Z (deflation with
// a fixed basis Z; E plays the role of the paper's T_r = U^T A U, eq. tau_mat).
//
// Storage: the basis is kept unnormalised -- column k holds `stored_k` and the
// normalised vector is v_k = vscale[k] * stored_k -- so no pass over memory is
// spent on normalisation; the scale is folded into the SpMV epilogue and into
// the coefficients of the vector updates.
//
// Every kernel reads the device control block first and returns at once when
// the solve (gate 1) or the current cycle (gate 2) has ended, so the host can
// enqueue a whole cycle without waiting.
#include <hip/hip_ext.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "internal.hpp"

namespace gm {

constexpr int kCT = 1024;   // threads of the coarse-solve kernels
__device__ void coarse_matvec(int R, const double* __restrict__ Einv, int trans, const double* t,
                              double* __restrict__ s, double* red);

// Deflation partials of one row block (fused Z^T y epilogue): for each of the
// block's slots l (deflation column bb_col[l]), the sum over the block's rows
// of z * y restricted to that column.  Wave sums per slot, one barrier, then
// the waves' sums in order; written to tpart[slot_pos[l]].
template <int NT, typename ACC>
__device__ __forceinline__ void block_slots(int l0, int l1, const int* __restrict__ bb_col,
                                            const int* __restrict__ slot_pos, int zc, ACC zvv,
                                            ACC yi, bool valid, int64_t row,
                                            const int* __restrict__ zrp, const int* __restrict__ zci,
                                            const double* __restrict__ zv, double* __restrict__ tpart,
                                            double (*sred)[kBlockColsMax]) {
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
    for (int l = l0; l < l1; ++l) {
        const int col = bb_col[l];
        GM_DCHECK(l1 - l0 <= kBlockColsMax, kDbgSlot);
        ACC c = 0;
        if (valid) {
            if (zc >= 0) {
                if (zc == col) c = zvv * yi;
            } else if (zc == -2) {
                for (int q = zrp[row]; q < zrp[row + 1]; ++q)
                    if (zci[q] == col) c += (ACC)zv[q] * yi;
                GM_DCHECK(zrp[row] <= zrp[row + 1], kDbgDeflCol);
            }
        }
        c = wave_sum(c);
        if (ln == 0) sred[wv][l - l0] = (double)c;
    }
    __syncthreads();
    for (int l = l0 + threadIdx.x; l < l1; l += NT) {
        double t = sred[0][l - l0];
#pragma unroll
        for (int q = 1; q < NT / kWave; ++q) t += sred[q][l - l0];
        tpart[slot_pos[l]] = t;
    }
    __syncthreads();
}

// ------------------------------------------------------------------- SpMV
// y = scale * A x, L lanes per row (row-per-group; L = 64 is row-per-wavefront).
template <int L, typename AT, typename XT, typename YT, typename ACC>
__global__ __launch_bounds__(kWG) void k_spmv(int n, const int* __restrict__ rowptr,
                                              const int* __restrict__ colind,
                                              const AT* __restrict__ vals,
                                              const XT* __restrict__ x,
                                              const double* __restrict__ scale_ptr,
                                              YT* __restrict__ y, const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    const int lane = threadIdx.x & (L - 1);
    constexpr int kRows = kWG / L;
    const ACC scale = scale_ptr ? (ACC)(*scale_ptr) : (ACC)1;
    for (int row = blockIdx.x * kRows + threadIdx.x / L; row < n; row += gridDim.x * kRows) {
        const int k0 = rowptr[row], k1 = rowptr[row + 1];
        ACC s = 0;
        for (int k = k0 + lane; k < k1; k += L) {
            GM_DCHECK(colind[k] >= 0 && colind[k] < n, kDbgCsrCol);
            s += (ACC)vals[k] * (ACC)ld_f(x + colind[k]);
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
        if (lane == 0) y[row] = (YT)(s * scale);
    }
}

// LDS-staged CSR stream (one row per thread, RB rows per block): the block's
// contiguous range of values and column indices is first copied to LDS with
// coalesced loads, then each thread forms its row's dot product from LDS and
// gathers x.  MODE 0: y = scale * A x.  MODE 1: y = b - A x and per-block
// partial sums of ||y||^2 into part[slot*NB + block].  Blocks whose entries do
// not fit the staging buffer read their rows directly.
// ZT: also the deflation partials of Z^T y -- one block sum per deflation
// column the row block reaches (bb_col), written to tpart[slot] (fixed order).
template <int RB, int MODE, bool ZT, typename AT, typename XT, typename BT, typename YT, typename ACC>
__global__ __launch_bounds__(RB) void k_spmv_stream(int n, const int* __restrict__ rowptr,
                                                    const int* __restrict__ colind,
                                                    const AT* __restrict__ vals,
                                                    const XT* __restrict__ x,
                                                    const double* __restrict__ scale_ptr,
                                                    const BT* __restrict__ b, YT* __restrict__ y,
                                                    double* __restrict__ part, int slot, int NB,
                                                    const int* __restrict__ zrp,
                                                    const int* __restrict__ zci,
                                                    const double* __restrict__ zv,
                                                    const int* __restrict__ bb_ptr,
                                                    const int* __restrict__ bb_col,
                                                    const int* __restrict__ slot_pos,
                                                    const int* __restrict__ zc1,
                                                    const double* __restrict__ zv1,
                                                    double* __restrict__ tpart,
                                                    const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    constexpr int CAP = 4096;
    __shared__ AT sv[CAP];
    __shared__ int sc[CAP];
    __shared__ ACC red[RB / kWave];
    __shared__ double sred[ZT ? RB / kWave : 1][kBlockColsMax];
    const ACC scale = (MODE == 0 && scale_ptr) ? (ACC)(*scale_ptr) : (ACC)1;
    ACC nrm = 0;
    for (int64_t r0 = (int64_t)blockIdx.x * RB; r0 < n; r0 += (int64_t)gridDim.x * RB) {
        const int64_t rend = min((int64_t)n, r0 + RB);
        const int k0 = rowptr[r0];
        const int cnt = rowptr[rend] - k0;
        const int64_t row = r0 + threadIdx.x;
        int zc = -1;
        ACC zvv = 0;
        if (ZT && row < rend) {
            zc = zc1[row];
            zvv = (ACC)zv1[row];
        }
        ACC acc = 0;
        if (cnt <= CAP) {
            for (int q = threadIdx.x; q < cnt; q += RB) {
                sv[q] = vals[k0 + q];
                sc[q] = colind[k0 + q];
            }
            __syncthreads();
            if (row < rend) {
                const int a = rowptr[row] - k0, e = rowptr[row + 1] - k0;
                for (int q = a; q < e; ++q) {
                    GM_DCHECK(sc[q] >= 0 && sc[q] < n, kDbgCsrCol);
                    acc += (ACC)sv[q] * (ACC)ld_f(x + sc[q]);
                }
            }
            __syncthreads();
        } else if (row < rend) {
            for (int k = rowptr[row]; k < rowptr[row + 1]; ++k) {
                GM_DCHECK(colind[k] >= 0 && colind[k] < n, kDbgCsrCol);
                acc += (ACC)vals[k] * (ACC)ld_f(x + colind[k]);
            }
        }
        ACC yi = 0;
        if (row < rend) {
            if (MODE == 0) {
                const YT v = (YT)(acc * scale);
                y[row] = v;
                yi = (ACC)v;
            } else {
                const YT v = (YT)((ACC)b[row] - acc);
                y[row] = v;
                yi = (ACC)v;
                nrm += yi * yi;
            }
        }
        if (ZT) {
            const int64_t blk = r0 / RB;
            block_slots<RB, ACC>(bb_ptr[blk], bb_ptr[blk + 1], bb_col, slot_pos, zc, zvv, yi,
                                 row < rend, row, zrp, zci, zv, tpart, sred);
        }
    }
    if (MODE == 1) {
        const ACC t = block_sum_n<RB>(nrm, red);
        if (threadIdx.x == 0) part[(int64_t)slot * NB + blockIdx.x] = (double)t;
    }
}

// One matrix entry (offset or value): plain, or with the non-temporal hint.
template <bool STREAM, typename T>
__device__ __forceinline__ T ld_mat(const T* p) {
    if constexpr (STREAM) return __builtin_nontemporal_load(p);
    else return *p;
}

// WMAX of a fixed-width instance whose matrix entries carry the non-temporal
// hint (the matrix does not fit in the last-level cache): kSellStreamW + width.
constexpr int kSellStreamW = 1000;

// Sliced-ELL SpMV: one wavefront per 64-position slice, NT positions per
// block, so every load instruction reads 64 consecutive entries of one slice
// column; position p holds row perm[p] (rows sorted within 256-row blocks) or
// p.  MODE / ZT as for the stream kernel (ZT needs NT = 256, the row blocks
// of the slots: a block's positions hold the same rows in either order).
template <int MODE, bool ZT, int WMAX, int NT, typename AT, typename XT, typename BT, typename YT,
          typename ACC>
__global__ __launch_bounds__(NT) void k_spmv_sell(int n, const int* __restrict__ off,
                                                   const int* __restrict__ perm, int wuni,
                                                   const short* __restrict__ scol,
                                                   const AT* __restrict__ sval,
                                                   const XT* __restrict__ x,
                                                   const double* __restrict__ scale_ptr,
                                                   const BT* __restrict__ b, YT* __restrict__ y,
                                                   double* __restrict__ part, int slot, int NB,
                                                   const int* __restrict__ zrp,
                                                   const int* __restrict__ zci,
                                                   const double* __restrict__ zv,
                                                   const int* __restrict__ bb_ptr,
                                                   const int* __restrict__ bb_col,
                                                   const int* __restrict__ slot_pos,
                                                   const int* __restrict__ zc1,
                                                   const double* __restrict__ zv1,
                                                   double* __restrict__ tpart, const Ctrl* ctrl,
                                                   int gate) {
    static_assert(!ZT || NT == kWG, "fused slots need 256-row blocks");
    __shared__ ACC red[NT / kWave];
    __shared__ double sred[ZT ? NT / kWave : 1][kBlockColsMax];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    // The control block is requested here and tested after the first row
    // block's independent loads are in flight (the test is uniform).
    const bool stopped = gated(ctrl, gate);
    const ACC scale = (MODE == 0 && scale_ptr) ? (ACC)(*scale_ptr) : (ACC)1;
    ACC nrm = 0;
    // Die-contiguous row blocks: the stencil's vector entries stay in one L2.
    const int64_t b0 = xcd_block(blockIdx.x, gridDim.x);
    for (int64_t r0 = b0 * NT; r0 < n; r0 += (int64_t)gridDim.x * NT) {
        const int64_t pos = r0 + threadIdx.x;
        // Beyond n the position is its own (invalid) row.
        const int64_t row = perm && pos < n ? (int64_t)perm[pos] : pos;
        const int64_t sl = r0 / kWave + wv;
        // Loads that do not depend on each other: slice bounds (none when every
        // slice has the same width), the row's Z entry, b, the block's slots.
        int q0, w;
        if (wuni > 0) {
            q0 = (int)(sl * wuni * kWave);
            w = wuni;
        } else {
            // The slice bounds are the same in every lane of the wavefront.
            q0 = __builtin_amdgcn_readfirstlane(off[sl]);
            w = (__builtin_amdgcn_readfirstlane(off[sl + 1]) - q0) / kWave;
        }
        int zc = -1;
        ACC zvv = 0;
        if (ZT && row < n) {
            zc = zc1[row];
            zvv = (ACC)zv1[row];
        }
        ACC bv = 0;
        if (MODE == 1 && row < n) bv = (ACC)b[row];
        int l0 = 0, l1 = 0;
        if (ZT) {
            const int64_t blk = r0 / kWG;
            l0 = bb_ptr[blk];
            l1 = bb_ptr[blk + 1];
        }
        if (stopped) return;
        ACC acc = 0;
        if (row < n) {
            const int q = q0 + lane;
            const XT* __restrict__ xr = x + row;   // columns are stored as offsets from the row
            // Loads are branch-free (column index clamped to the slice's last
            // column, products past the width dropped by a select), so the
            // compiler can count outstanding loads exactly and never waits
            // for one gather before issuing the next.
            if (w > 0) {
                constexpr bool kFixStream = WMAX > kSellStreamW;
                constexpr int WF = kFixStream ? WMAX - kSellStreamW : WMAX;
                if constexpr (WF > 0) {
                    // Every slice is at most WMAX wide (the launch picks WMAX
                    // from the longest row): offsets and values of the whole
                    // row, then the gathers, then the products.
                    int cc[WF];
                    AT vv[WF];
#pragma unroll
                    for (int k = 0; k < WF; ++k) {
                        const int kk = min(k, w - 1);
                        cc[k] = ld_mat<kFixStream>(scol + q + kk * kWave);
                        vv[k] = ld_mat<kFixStream>(sval + q + kk * kWave);
                    }
                    ACC xv[WF];
#pragma unroll
                    for (int k = 0; k < WF; ++k) {
                        GM_DCHECK(row + cc[k] >= 0 && row + cc[k] < n, kDbgSellCol);
                        xv[k] = (ACC)ld_f(xr + cc[k]);
                    }
#pragma unroll
                    for (int k = 0; k < WF; ++k) acc += k < w ? (ACC)vv[k] * xv[k] : (ACC)0;
                } else {
                    // Rows of any length, in chunks of CH entries: the values
                    // and gathers of one chunk are issued, then the column
                    // offsets of the next, which stay in flight while the
                    // products of the first wait.  WMAX < 0: the matrix is
                    // larger than the last-level cache, so its offsets and
                    // values stream past it (non-temporal hint) and leave it
                    // to the input vector and the Krylov basis.
                    constexpr int CH = 8;
                    constexpr bool kStream = WMAX < 0;
                    int cc[CH];
#pragma unroll
                    for (int k = 0; k < CH; ++k) cc[k] = ld_mat<kStream>(scol + q + min(k, w - 1) * kWave);
                    for (int k0 = 0; k0 < w; k0 += CH) {
                        ACC xv[CH];
                        AT va[CH];
#pragma unroll
                        for (int k = 0; k < CH; ++k) {
                            GM_DCHECK(row + cc[k] >= 0 && row + cc[k] < n, kDbgSellCol);
                            va[k] = ld_mat<kStream>(sval + q + min(k0 + k, w - 1) * kWave);
                            xv[k] = (ACC)ld_f(xr + cc[k]);
                        }
#pragma unroll
                        for (int k = 0; k < CH; ++k)
                            cc[k] = ld_mat<kStream>(scol + q + min(k0 + CH + k, w - 1) * kWave);
#pragma unroll
                        for (int k = 0; k < CH; ++k)
                            acc += k0 + k < w ? (ACC)va[k] * xv[k] : (ACC)0;
                    }
                }
            }
        }
        ACC yi = 0;
        if (row < n) {
            if (MODE == 0) {
                const YT v = (YT)(acc * scale);
                y[row] = v;
                yi = (ACC)v;
            } else {
                const YT v = (YT)(bv - acc);
                y[row] = v;
                yi = (ACC)v;
                nrm += yi * yi;
            }
        }
        if (ZT)
            block_slots<NT, ACC>(l0, l1, bb_col, slot_pos, zc, zvv, yi, row < n, row, zrp, zci,
                                  zv, tpart, sred);
    }
    if (stopped) return;
    if (MODE == 1) {
        const ACC t = block_sum_n<NT>(nrm, red);
        if (threadIdx.x == 0) part[(int64_t)slot * NB + blockIdx.x] = (double)t;
    }
}

// s = E^{-1} t with t_a = sum of the slots of deflation column a, which are
// stored contiguously (tpart[ab_ptr[a] .. ab_ptr[a+1]), increasing row blocks).
// Column a goes to a run of SG consecutive threads (SG = the largest power of
// two with R * SG <= kCT); member g reads slots q0 + g, q0 + g + SG, ..., so
// neighbouring lanes read neighbouring slots and up to kSU loads per thread
// are in flight at once.  Each thread adds its loads in order, the run adds
// its members by butterfly (within a wavefront) and then by wavefront in
// order.  The slot ranges, this thread's E^{-1} entries and the control
// block are requested together before any slot is read.
__global__ __launch_bounds__(kCT) void k_coarse_slots(int R, const int* __restrict__ ab_ptr,
                                                      const double* __restrict__ tpart,
                                                      const double* __restrict__ Einv, int trans,
                                                      double* __restrict__ s, const Ctrl* ctrl,
                                                      int gate) {
    __shared__ double t[kMaxR];
    __shared__ double red[kCT];
    int SG = kCT;
    while (SG * R > kCT) SG >>= 1;
    const int col = threadIdx.x / SG, g = threadIdx.x % SG;
    int q0 = 0, q1 = 0;
    if (col < R) {
        q0 = ab_ptr[col];
        q1 = ab_ptr[col + 1];
        GM_DCHECK(0 <= q0 && q0 <= q1, kDbgSlot);
    }
    // E^{-1} entries of this thread (same split as coarse_matvec).
    const int G = max(1, kCT / R);
    const int grp = threadIdx.x / R, a = threadIdx.x % R;
    constexpr int kEmax = 8;   // prefetched entries per thread (R up to about 90)
    double ev[kEmax];
    const int espan = (R + G - 1) / G;
    const int ea0 = grp * espan, ea1 = (grp < G) ? min(R, ea0 + espan) : ea0;
    const bool pre = espan <= kEmax;
    if (pre) {
#pragma unroll
        for (int u = 0; u < kEmax; ++u) {
            const int aa = ea0 + u;
            ev[u] = (aa < ea1) ? (trans ? Einv[(int64_t)a * R + aa] : Einv[(int64_t)aa * R + a]) : 0.0;
        }
    }
    if (gated(ctrl, gate)) return;
    constexpr int kSU = 16;
    double acc = 0;
    for (int qb = q0 + g; qb < q1; qb += kSU * SG) {
        double v[kSU];
#pragma unroll
        for (int u = 0; u < kSU; ++u) {
            const int q = qb + u * SG;
            v[u] = q < q1 ? tpart[q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSU; ++u) acc += v[u];
    }
    // Runs of SG <= kWave lanes are aligned inside a wavefront, so xor
    // partners below SG stay in the run.
    const int lw = min(SG, kWave);
    for (int o = lw / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (SG <= kWave) {
        if (g == 0 && col < R) t[col] = acc;
    } else {
        const int wv = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) red[wv] = acc;
        __syncthreads();
        if (g == 0 && col < R) {
            double v = red[wv];
            for (int q = 1; q < SG / kWave; ++q) v += red[wv + q];
            t[col] = v;
        }
    }
    __syncthreads();
    if (!pre) {
        coarse_matvec(R, Einv, trans, t, s, red);
        return;
    }
    // s = E^{-1} t with the prefetched entries (same split and order as
    // coarse_matvec).
    double v = 0;
    if (grp < G) {
#pragma unroll
        for (int u = 0; u < kEmax; ++u)
            if (ea0 + u < ea1) v += ev[u] * t[ea0 + u];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < R) {
        double r = red[threadIdx.x];
        for (int q = 1; q < G; ++q) r += red[q * R + threadIdx.x];
        s[threadIdx.x] = r;
    }
}

// r = b - A x (x in FP64), plus per-workgroup partial sums of ||r||^2 into
// part[slot*NB + block].
template <int L, typename AT, typename BT, typename RT, typename ACC>
__global__ __launch_bounds__(kWG) void k_residual(int n, const int* __restrict__ rowptr,
                                                  const int* __restrict__ colind,
                                                  const AT* __restrict__ vals,
                                                  const double* __restrict__ x,
                                                  const BT* __restrict__ b, RT* __restrict__ r,
                                                  double* __restrict__ part, int slot, int NB,
                                                  const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ ACC red[kWG / kWave];
    const int lane = threadIdx.x & (L - 1);
    constexpr int kRows = kWG / L;
    ACC nrm = 0;
    for (int row = blockIdx.x * kRows + threadIdx.x / L; row < n; row += gridDim.x * kRows) {
        const int k0 = rowptr[row], k1 = rowptr[row + 1];
        ACC s = 0;
        for (int k = k0 + lane; k < k1; k += L) s += (ACC)vals[k] * (ACC)x[colind[k]];
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
        if (lane == 0) {
            const ACC ri = (ACC)b[row] - s;
            r[row] = (RT)ri;
            nrm += ri * ri;
        }
    }
    const ACC t = block_sum(nrm, red);
    if (threadIdx.x == 0) part[(int64_t)slot * NB + blockIdx.x] = (double)t;
}

// ------------------------------------------------------ deflation (per step)
// Partial sums of t = Z^T y over chunks of the rows of Z^T (CSR of Z^T):
// block (a, c) sums entries [ztrp[a] + c*CH, ...) in index order.
template <typename YT>
__global__ __launch_bounds__(kWG) void k_zt(int R, int MC, int CH, const int* __restrict__ ztrp,
                                            const int* __restrict__ ztci,
                                            const double* __restrict__ ztv,
                                            const YT* __restrict__ y, double* __restrict__ tpart,
                                            const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ double red[kWG / kWave];
    const int a = blockIdx.x / MC, c = blockIdx.x % MC;
    const int q0 = ztrp[a] + c * CH;
    const int q1 = min(ztrp[a + 1], q0 + CH);
    double s = 0;
    for (int q = q0 + threadIdx.x; q < q1; q += kWG) s += ztv[q] * (double)y[ztci[q]];
    s = block_sum(s, red);
    if (threadIdx.x == 0) tpart[(int64_t)a * MC + c] = s;
}

// s = E^{-1} t (or E^{-T} t for the adjoint, `trans`), with the explicit
// inverse from setup stored column-major (Einv[i][a] at Einv[a*R + i]).  All
// kCT threads take part: output i is split over G = kCT / R thread groups, each
// summing a contiguous range of a, then the G partial sums are added in order.
__device__ void coarse_matvec(int R, const double* __restrict__ Einv, int trans, const double* t,
                              double* __restrict__ s, double* red /* kCT */) {
    const int G = max(1, kCT / R);
    const int grp = threadIdx.x / R, i = threadIdx.x % R;
    double acc = 0;
    if (grp < G) {
        const int span = (R + G - 1) / G;
        const int a0 = grp * span, a1 = min(R, a0 + span);
        if (!trans) {
#pragma unroll 8
            for (int a = a0; a < a1; ++a) acc += Einv[(int64_t)a * R + i] * t[a];
        } else {
#pragma unroll 8
            for (int a = a0; a < a1; ++a) acc += Einv[(int64_t)i * R + a] * t[a];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < R) {
        double v = red[threadIdx.x];
        for (int q = 1; q < G; ++q) v += red[q * R + threadIdx.x];
        s[threadIdx.x] = v;
    }
}

// s = E^{-1} t with t = sum over chunks of tpart (fixed order).
__global__ __launch_bounds__(kCT) void k_coarse(int R, int MC, const double* __restrict__ tpart,
                                                const double* __restrict__ Einv, int trans,
                                                double* __restrict__ s, const Ctrl* ctrl,
                                                int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ double t[kMaxR];
    __shared__ double red[kCT];
    for (int a = threadIdx.x; a < R; a += kCT) {
        double acc = 0;
        for (int c = 0; c < MC; ++c) acc += tpart[(int64_t)a * MC + c];
        t[a] = acc;
    }
    __syncthreads();
    coarse_matvec(R, Einv, trans, t, s, red);
}

// ------------------------------------------------------------- CGS2 passes
// Lane layout: each lane moves 16 bytes of a basis column per load, i.e. a
// tile of R = 16 / sizeof(VT) consecutive rows (2 FP64, 4 FP32, 8 FP16).  T
// consecutive lanes share one tile; lane `sub` owns basis columns
// k = sub, sub + T, ... so it keeps JMAX / T raw 16-byte tiles and as many dot
// accumulators in registers.  Vectors are padded with zeros to a multiple of
// 64 entries, so whole tiles are read and written; only the deflation rows
// are bounded by n.

template <typename T, int R, typename ACC>
__device__ __forceinline__ void load_tile(const T* __restrict__ p, ACC (&out)[R]) {
    constexpr int NC = (R * (int)sizeof(T) + 15) / 16;
    T tmp[NC * 16 / sizeof(T)];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint4 u = reinterpret_cast<const uint4*>(p)[c];
        __builtin_memcpy(reinterpret_cast<char*>(tmp) + 16 * c, &u, 16);
    }
#pragma unroll
    for (int e = 0; e < R; ++e) out[e] = (ACC)ld_f(tmp + e);
}

template <typename T, int R, typename ACC>
__device__ __forceinline__ void store_tile(T* __restrict__ p, const ACC (&in)[R]) {
    constexpr int NC = (R * (int)sizeof(T) + 15) / 16;
    T tmp[NC * 16 / sizeof(T)];
#pragma unroll
    for (int e = 0; e < R; ++e) st_v(tmp + e, in[e]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        uint4 u;
        __builtin_memcpy(&u, reinterpret_cast<const char*>(tmp) + 16 * c, 16);
        reinterpret_cast<uint4*>(p)[c] = u;
    }
}

// Exactly R consecutive entries (R * sizeof(T) = 2, 4, 8 or a multiple of 16
// bytes, at an address aligned to that size or to 16 bytes).
template <typename T, int R>
struct RowBytes {
    static constexpr int B = R * (int)sizeof(T);
    static_assert(B == 2 || B == 4 || B == 8 || B % 16 == 0, "row group of 2, 4, 8 or 16k bytes");
};

template <typename T, int R, typename ACC>
__device__ __forceinline__ void load_rows(const T* __restrict__ p, ACC (&out)[R]) {
    constexpr int B = RowBytes<T, R>::B;
    T tmp[R];
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int c = 0; c < B / 16; ++c) {
            const uint4 u = reinterpret_cast<const uint4*>(p)[c];
            __builtin_memcpy(reinterpret_cast<char*>(tmp) + 16 * c, &u, 16);
        }
    } else if constexpr (B == 8) {
        const uint2 u = *reinterpret_cast<const uint2*>(p);
        __builtin_memcpy(tmp, &u, 8);
    } else if constexpr (B == 4) {
        const unsigned int u = *reinterpret_cast<const unsigned int*>(p);
        __builtin_memcpy(tmp, &u, 4);
    } else {
        const unsigned short u = *reinterpret_cast<const unsigned short*>(p);
        __builtin_memcpy(tmp, &u, 2);
    }
#pragma unroll
    for (int e = 0; e < R; ++e) out[e] = (ACC)ld_f(tmp + e);
}

template <typename T, int R, typename ACC>
__device__ __forceinline__ void store_rows(T* __restrict__ p, const ACC (&in)[R]) {
    constexpr int B = RowBytes<T, R>::B;
    T tmp[R];
#pragma unroll
    for (int e = 0; e < R; ++e) st_v(tmp + e, in[e]);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int c = 0; c < B / 16; ++c) {
            uint4 u;
            __builtin_memcpy(&u, reinterpret_cast<const char*>(tmp) + 16 * c, 16);
            reinterpret_cast<uint4*>(p)[c] = u;
        }
    } else if constexpr (B == 8) {
        uint2 u;
        __builtin_memcpy(&u, tmp, 8);
        *reinterpret_cast<uint2*>(p) = u;
    } else if constexpr (B == 4) {
        unsigned int u;
        __builtin_memcpy(&u, tmp, 4);
        *reinterpret_cast<unsigned int*>(p) = u;
    } else {
        unsigned short u;
        __builtin_memcpy(&u, tmp, 2);
        *reinterpret_cast<unsigned short*>(p) = u;
    }
}

template <int R>
__device__ __forceinline__ void load_ints(const int* __restrict__ p, int (&out)[R]) {
    if constexpr (R == 2) {
        const uint2 u = *reinterpret_cast<const uint2*>(p);
        out[0] = (int)u.x;
        out[1] = (int)u.y;
    } else {
#pragma unroll
        for (int c = 0; c < R / 4; ++c) {
            const uint4 u = reinterpret_cast<const uint4*>(p)[c];
            out[4 * c] = (int)u.x;
            out[4 * c + 1] = (int)u.y;
            out[4 * c + 2] = (int)u.z;
            out[4 * c + 3] = (int)u.w;
        }
    }
}

template <typename VT, typename ACC>
__device__ __forceinline__ ACC raw_at(const uint4& u, int e) {
    VT tmp[16 / sizeof(VT)];
    __builtin_memcpy(tmp, &u, 16);
    return (ACC)ld_f(tmp + e);
}

// Cross-lane moves inside a row of 16 lanes (DPP): quad_perm [1,0,3,2] (0xB1),
// quad_perm [2,3,0,1] (0x4E), half-row mirror (0x141), row mirror (0x140).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the T consecutive lanes of a tile group (T <= 16, groups aligned
// to T); every lane of the group gets the same value (the pairings are
// symmetric, so both partners add the same two operands).
template <int T, typename ACC>
__device__ __forceinline__ ACC group_sum(ACC v) {
    static_assert(T >= 1 && T <= 16 && (T & (T - 1)) == 0, "tile group of 1..16 lanes");
    if constexpr (T >= 2) v += dpp_mov<0xB1>(v);
    if constexpr (T >= 4) v += dpp_mov<0x4E>(v);
    if constexpr (T >= 8) v += dpp_mov<0x141>(v);
    if constexpr (T >= 16) v += dpp_mov<0x140>(v);
    return v;
}

// Basis tiles of one lane: tile q holds column k = sub + q*T at rows
// i0 .. i0+R-1.  Every tile slot is filled (branch-free code): slots past the
// last column re-read column nv-1 (an address another lane of the same wave
// reads, so no extra memory traffic) and carry coefficient 0; their dot
// accumulators are never stored.  Requires nv >= 1.
// A basis that outgrows the 256 MB last-level cache (FP64 from about a
// million rows, FP16 from about four million) keeps its first `keep` columns
// (as many as fit there beside the matrix and the work vectors; chosen per
// plan and precision) on plain loads, so they stay cached for both sweeps of
// every step; the tile slots whose columns reach past them carry the
// non-temporal hint, so the rest of the basis streams through without
// displacing what the next step reads again (non-temporal streaming reads
// also run about 10% faster than plain ones on this part).  The test is
// uniform per slot q.
template <int JT, int T, typename VT>
__device__ __forceinline__ void load_cols(const VT* __restrict__ V, int64_t ldv, int nv, int sub,
                                          int64_t i0, int keep, uint4 (&raw)[JT]) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < JT; ++q) {
        const int k = min(sub + q * T, nv - 1);
        if ((q + 1) * T > keep) {
            const u32x4 t = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(V + k * ldv + i0));
            raw[q] = make_uint4(t.x, t.y, t.z, t.w);
        } else {
            raw[q] = *reinterpret_cast<const uint4*>(V + k * ldv + i0);
        }
    }
}

// Coefficients of a lane's columns, staged through LDS (c_l holds JMAX
// entries, zero from nv on).
template <int JMAX, int T, typename ACC>
__device__ __forceinline__ void stage_coef(const double* __restrict__ coef, int nv, ACC* c_l,
                                           int sub, ACC (&cr)[JMAX / T]) {
    for (int k = threadIdx.x; k < JMAX; k += kWG) c_l[k] = k < nv ? (ACC)coef[k] : (ACC)0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < JMAX / T; ++q) cr[q] = c_l[sub + q * T];
}

// sum_q cr[q] * (row e of tile q), over the lane's columns, then over the group.
template <int JT, int T, typename VT, typename ACC>
__device__ __forceinline__ ACC combine_row(const uint4 (&raw)[JT], const ACC (&cr)[JT], int e) {
    ACC u = 0;
#pragma unroll
    for (int q = 0; q < JT; ++q) u += raw_at<VT, ACC>(raw[q], e) * cr[q];
    return group_sum<T>(u);
}

// acc[q] += (tile q) . x over the tile's rows.
template <int JT, int T, int R, typename VT, typename ACC>
__device__ __forceinline__ void accumulate_dots(const uint4 (&raw)[JT], const ACC (&x)[R],
                                                ACC (&acc)[JT]) {
#pragma unroll
    for (int q = 0; q < JT; ++q) {
        ACC t = 0;
#pragma unroll
        for (int e = 0; e < R; ++e) t += raw_at<VT, ACC>(raw[q], e) * x[e];
        acc[q] += t;
    }
}

// w = y - (A Z) s for one tile, from the two-entry row copy of A Z (pairs
// (column, value) per row, -1 / 0 where absent); rows with more entries are
// marked -2 and fall back to the CSR copy.  The common rows are handled
// without branches or dependent loads.
template <int RT, typename AZT, typename ACC>
__device__ __forceinline__ void deflate_tile(int64_t i0, const int* __restrict__ azrp,
                                             const int* __restrict__ azci,
                                             const AZT* __restrict__ azv,
                                             const int* __restrict__ azc2,
                                             const AZT* __restrict__ azv2, const ACC* s_l,
                                             ACC (&u)[RT]) {
    int ac[2 * RT];
    ACC av[2 * RT];
    load_ints<2 * RT>(azc2 + 2 * i0, ac);
    load_rows<AZT, 2 * RT, ACC>(azv2 + 2 * i0, av);
    bool multi = false;
#pragma unroll
    for (int e = 0; e < RT; ++e) {
        GM_DCHECK(ac[2 * e] >= -2 && ac[2 * e] < kMaxR && ac[2 * e + 1] >= -1 && ac[2 * e + 1] < kMaxR,
                  kDbgDeflCol);
        u[e] -= av[2 * e] * s_l[max(ac[2 * e], 0)] + av[2 * e + 1] * s_l[max(ac[2 * e + 1], 0)];
        multi |= ac[2 * e] == -2;
    }
    if (multi) {
#pragma unroll
        for (int e = 0; e < RT; ++e) {
            if (ac[2 * e] == -2) {
                const int64_t i = i0 + e;
                for (int q = azrp[i]; q < azrp[i + 1]; ++q) {
                    GM_DCHECK(azci[q] >= 0 && azci[q] < kMaxR, kDbgDeflCol);
                    u[e] -= (ACC)azv[q] * s_l[azci[q]];
                }
            }
        }
    }
}

// Writes the workgroup sums of the per-lane accumulators acc[q] (column
// k = sub + q*T) and of accn (norm slot) to part.  Fixed order: butterfly
// over the lanes with equal `sub`, then waves in order.
template <int JMAX, int T, typename ACC>
__device__ __forceinline__ void store_partials(const ACC (&acc)[JMAX / T], ACC accn, int nv,
                                               ACC (*red)[JMAX + 1], double* part, int nslot,
                                               int NB) {
    constexpr int JT = JMAX / T;
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
    const int sub = ln & (T - 1);
#pragma unroll
    for (int q = 0; q < JT; ++q) {
        if (q * T < nv) {
            ACC t = acc[q];
#pragma unroll
            for (int o = kWave / 2; o >= T; o >>= 1) t += __shfl_xor(t, o, kWave);
            const int k = sub + q * T;
            if (ln < T && k < nv) red[wv][k] = t;
        }
    }
    {
        ACC t = wave_sum(accn);
        if (ln == 0) red[wv][JMAX] = t;
    }
    __syncthreads();
    const int tk = threadIdx.x;
    if (tk < nv || tk == JMAX) {
        ACC t = red[0][tk];
#pragma unroll
        for (int q = 1; q < kWG / kWave; ++q) t += red[q][tk];
        const int slot = (tk == JMAX) ? nslot : tk;
        part[(int64_t)slot * NB + blockIdx.x] = (double)t;
    }
}

// Pass 1: w = y - (A Z) s  (deflation, compact CSR of A Z), then partial
// dots stored_k^T w for k < nv and ||w||^2 (norm slot).  nv = 0 gives the
// deflated restart vector p = P r and its norm.
template <int JMAX, int T, typename VT, typename WT, typename AZT, typename ACC>
__global__ __launch_bounds__(kWG) void k_pass1(int n, int64_t ldv, const VT* __restrict__ V, int nv,
                                               const WT* __restrict__ y,
                                               const int* __restrict__ azrp,
                                               const int* __restrict__ azci,
                                               const AZT* __restrict__ azv,
                                               const int* __restrict__ azc2,
                                               const AZT* __restrict__ azv2,
                                               const double* __restrict__ s, int R,
                                               WT* __restrict__ w, double* __restrict__ part,
                                               int nslot, int NB, const Ctrl* ctrl, int gate, int keep) {
    constexpr int JT = JMAX / T;
    constexpr int RT = 16 / sizeof(VT);
    __shared__ ACC s_l[kMaxR];
    __shared__ ACC red[kWG / kWave][JMAX + 1];
    for (int a = threadIdx.x; a < R; a += kWG) s_l[a] = (ACC)s[a];
    __syncthreads();
    // Tested after the staging loads so the two requests overlap (uniform).
    if (gated(ctrl, gate)) return;
    const int sub = threadIdx.x & (T - 1);
    ACC acc[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) acc[q] = 0;
    ACC accn = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T) * RT;
    for (int64_t i0 = (((int64_t)blockIdx.x * kWG + threadIdx.x) / T) * RT; i0 < n; i0 += stride) {
        uint4 raw[JT];
        if (nv > 0) load_cols<JT, T, VT>(V, ldv, nv, sub, i0, keep, raw);
        ACC wv[RT];
        load_tile<WT, RT, ACC>(y + i0, wv);
        if (R > 0) deflate_tile<RT, AZT, ACC>(i0, azrp, azci, azv, azc2, azv2, s_l, wv);
        if (sub == 0) {
            store_tile<WT, RT, ACC>(w + i0, wv);
#pragma unroll
            for (int e = 0; e < RT; ++e) accn += wv[e] * wv[e];
        }
        if (nv > 0) accumulate_dots<JT, T, RT, VT, ACC>(raw, wv, acc);
    }
    store_partials<JMAX, T, ACC>(acc, accn, nv, red, part, nslot, NB);
}

// Pass 2: w -= sum_k stored_k c_k (first Gram-Schmidt update), then partial
// dots stored_k^T w and ||w||^2 of the updated vector.
template <int JMAX, int T, typename VT, typename WT, typename ACC>
__global__ __launch_bounds__(kWG) void k_pass2(int n, int64_t ldv, const VT* __restrict__ V, int nv,
                                               WT* __restrict__ w, const double* __restrict__ coef,
                                               double* __restrict__ part, int nslot, int NB,
                                               const Ctrl* ctrl, int gate, int keep) {
    constexpr int JT = JMAX / T;
    constexpr int RT = 16 / sizeof(VT);
    __shared__ ACC c_l[JMAX];
    __shared__ ACC red[kWG / kWave][JMAX + 1];
    const int sub = threadIdx.x & (T - 1);
    ACC cr[JT];
    stage_coef<JMAX, T, ACC>(coef, nv, c_l, sub, cr);
    if (gated(ctrl, gate)) return;   // after the staging loads (uniform)
    ACC acc[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) acc[q] = 0;
    ACC accn = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T) * RT;
    for (int64_t i0 = (((int64_t)blockIdx.x * kWG + threadIdx.x) / T) * RT; i0 < n; i0 += stride) {
        uint4 raw[JT];
        load_cols<JT, T, VT>(V, ldv, nv, sub, i0, keep, raw);
        ACC wv[RT];
        load_tile<WT, RT, ACC>(w + i0, wv);
#pragma unroll
        for (int e = 0; e < RT; ++e) wv[e] -= combine_row<JT, T, VT, ACC>(raw, cr, e);
        if (sub == 0) {
            store_tile<WT, RT, ACC>(w + i0, wv);
#pragma unroll
            for (int e = 0; e < RT; ++e) accn += wv[e] * wv[e];
        }
        accumulate_dots<JT, T, RT, VT, ACC>(raw, wv, acc);
    }
    store_partials<JMAX, T, ACC>(acc, accn, nv, red, part, nslot, NB);
}

// Pass 3: w -= sum_k stored_k c_k (second update); the result, times the
// storage scale sigma, becomes basis column nv; partial sums of ||w||^2.
template <int JMAX, int T, typename VT, typename WT, typename ACC>
__global__ __launch_bounds__(kWG) void k_pass3(int n, int64_t ldv, VT* __restrict__ V, int nv,
                                               const WT* __restrict__ w,
                                               const double* __restrict__ coef,
                                               const double* __restrict__ sigma,
                                               double* __restrict__ part, int nslot, int NB,
                                               const Ctrl* ctrl, int gate, int keep) {
    constexpr int JT = JMAX / T;
    constexpr int RT = 16 / sizeof(VT);
    __shared__ ACC c_l[JMAX];
    __shared__ ACC red[kWG / kWave];
    const int sub = threadIdx.x & (T - 1);
    ACC cr[JT];
    stage_coef<JMAX, T, ACC>(coef, nv, c_l, sub, cr);
    if (gated(ctrl, gate)) return;   // after the staging loads (uniform)
    const ACC sg = (ACC)(*sigma);
    VT* __restrict__ vout = V + nv * ldv;
    ACC accn = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T) * RT;
    for (int64_t i0 = (((int64_t)blockIdx.x * kWG + threadIdx.x) / T) * RT; i0 < n; i0 += stride) {
        uint4 raw[JT];
        load_cols<JT, T, VT>(V, ldv, nv, sub, i0, keep, raw);
        ACC wv[RT];
        load_tile<WT, RT, ACC>(w + i0, wv);
#pragma unroll
        for (int e = 0; e < RT; ++e) wv[e] -= combine_row<JT, T, VT, ACC>(raw, cr, e);
        if (sub == 0) {
            ACC ov[RT];
#pragma unroll
            for (int e = 0; e < RT; ++e) {
                ov[e] = wv[e] * sg;
                accn += wv[e] * wv[e];
            }
            store_tile<VT, RT, ACC>(vout + i0, ov);
        }
    }
    const ACC t = block_sum(accn, red);
    if (threadIdx.x == 0) part[(int64_t)nslot * NB + blockIdx.x] = (double)t;
}

// ------------------------------------------- two-pass CGS2, lagged normalisation
// Step j (>= 1) of the lagged variant starts from the previous step's
// once-projected vector w1 = w_{j-1} - V h1 (not yet re-orthogonalised or
// normalised), its second-projection coefficients h2 and the estimate
// hn = ||w1 - V h2|| = sqrt(||w1||^2 - ||h2||^2).  The SpMV runs on w1:
// u = A w1.  This pass then, in one sweep over V_{0..j-1}:
//   w2 = w1 - V h2                       (second Gram-Schmidt update of w1),
//   v_j = w2 / hn                        (stored as sigma * w2),
//   w_j = P A v_j = (P u - sum_l v_l c_l - w2 h2_{j-1}) / hn,
// where P A V = V Hbar (the Arnoldi relation) gives P A (V h2) = V (Hbar h2),
// c = Hbar h2 restricted to rows l < j, and the last row's term is
// hn h2_{j-1} v_j = w2 h2_{j-1}; then the partial dots of w_j with v_0..v_j
// and ||w_j||^2.  So each step sweeps the basis twice instead of three times.
// lag[0] = h2_{j-1}, lag[1] = 1/hn, lag[2] = sigma (storage scale of v_j).
template <int JMAX, int T, typename VT, typename WT, typename AZT, typename ACC>
__global__ __launch_bounds__(kWG) void k_pass1_lag(int n, int64_t ldv, VT* __restrict__ V, int nvr,
                                                   WT* __restrict__ w, const WT* __restrict__ y,
                                                   const int* __restrict__ azrp,
                                                   const int* __restrict__ azci,
                                                   const AZT* __restrict__ azv,
                                                   const int* __restrict__ azc2,
                                                   const AZT* __restrict__ azv2,
                                                   const double* __restrict__ s, int R,
                                                   const double* __restrict__ coef2,
                                                   const double* __restrict__ cc,
                                                   const double* __restrict__ lag,
                                                   double* __restrict__ part, int nslot, int NB,
                                                   const Ctrl* ctrl, int gate, int keep) {
    constexpr int JT = JMAX / T;
    constexpr int RT = 16 / sizeof(VT);
    __shared__ ACC s_l[kMaxR];
    __shared__ ACC c2_l[JMAX], cc_l[JMAX];
    __shared__ ACC red[kWG / kWave][JMAX + 2];
    for (int a = threadIdx.x; a < R; a += kWG) s_l[a] = (ACC)s[a];
    const int sub = threadIdx.x & (T - 1);
    ACC c2r[JT], ccr[JT];
    for (int k = threadIdx.x; k < JMAX; k += kWG) cc_l[k] = k < nvr ? (ACC)cc[k] : (ACC)0;
    stage_coef<JMAX, T, ACC>(coef2, nvr, c2_l, sub, c2r);   // synchronises
#pragma unroll
    for (int q = 0; q < JT; ++q) ccr[q] = cc_l[sub + q * T];
    const ACC h2last = (ACC)lag[0], ihn = (ACC)lag[1], sg = (ACC)lag[2];
    if (gated(ctrl, gate)) return;   // after the staging loads (uniform)
    VT* __restrict__ vout = V + nvr * ldv;
    ACC acc[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) acc[q] = 0;
    ACC accn = 0, accd = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T) * RT;
    // With T > 1 lanes per tile, the first TS = min(T, RT) lanes of a tile
    // group each own RS = RT / TS of its rows: the owner alone loads their
    // w1, A w1 and A Z entries, deflates, forms and stores them and adds
    // them to the norms; the group then shares the new w rows (lane
    // shuffles) for the dot products.  With one lane per tile that lane
    // handles all RT rows.
    constexpr bool kSplit = T > 1;
    constexpr int TS = T < RT ? T : RT;
    constexpr int RS = kSplit ? RT / TS : RT;
    const bool owner = sub < TS;
    const int e0 = (kSplit && owner) ? sub * RS : 0;
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(T - 1);
    for (int64_t i0 = (((int64_t)blockIdx.x * kWG + threadIdx.x) / T) * RT; i0 < n; i0 += stride) {
        uint4 raw[JT];
        load_cols<JT, T, VT>(V, ldv, nvr, sub, i0, keep, raw);
        if constexpr (kSplit) {
            ACC w1[RS], u[RS];
#pragma unroll
            for (int r = 0; r < RS; ++r) w1[r] = u[r] = (ACC)0;
            if (owner) {
                load_rows<WT, RS, ACC>(w + i0 + e0, w1);
                load_rows<WT, RS, ACC>(y + i0 + e0, u);
                if (R > 0) deflate_tile<RS, AZT, ACC>(i0 + e0, azrp, azci, azv, azc2, azv2, s_l, u);
            }
            // Group sums for every row of the tile (all lanes take part), then
            // this lane's rows picked out with compile-time register indices.
            ACC a2o[RS], a3o[RS];
#pragma unroll
            for (int r = 0; r < RS; ++r) a2o[r] = a3o[r] = (ACC)0;
#pragma unroll
            for (int e = 0; e < RT; ++e) {
                const ACC a2 = combine_row<JT, T, VT, ACC>(raw, c2r, e);
                const ACC a3 = combine_row<JT, T, VT, ACC>(raw, ccr, e);
                const bool mine = (e / RS) == sub;
                a2o[e % RS] = mine ? a2 : a2o[e % RS];
                a3o[e % RS] = mine ? a3 : a3o[e % RS];
            }
            ACC svo[RS], wno[RS];
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                const ACC w2 = w1[r] - a2o[r];
                VT stv;
                st_v(&stv, w2 * sg);
                svo[r] = (ACC)ld_f(&stv);
                wno[r] = (u[r] - a3o[r] - w2 * h2last) * ihn;
                if (owner) {
                    accn += wno[r] * wno[r];
                    accd += svo[r] * wno[r];
                }
            }
            if (owner) {
                store_rows<VT, RS, ACC>(vout + i0 + e0, svo);
                store_rows<WT, RS, ACC>(w + i0 + e0, wno);
            }
            ACC wn[RT];
#pragma unroll
            for (int e = 0; e < RT; ++e) wn[e] = __shfl(wno[e % RS], gbase + e / RS, kWave);
            accumulate_dots<JT, T, RT, VT, ACC>(raw, wn, acc);
            continue;
        }
        ACC w1[RT], u[RT];
        load_tile<WT, RT, ACC>(w + i0, w1);
        load_tile<WT, RT, ACC>(y + i0, u);
        if (R > 0) deflate_tile<RT, AZT, ACC>(i0, azrp, azci, azv, azc2, azv2, s_l, u);
        ACC sv[RT], wn[RT];
#pragma unroll
        for (int e = 0; e < RT; ++e) {
            const ACC a2 = combine_row<JT, T, VT, ACC>(raw, c2r, e);
            const ACC a3 = combine_row<JT, T, VT, ACC>(raw, ccr, e);
            const ACC w2 = w1[e] - a2;
            VT stv;
            st_v(&stv, w2 * sg);
            sv[e] = (ACC)ld_f(&stv);
            wn[e] = (u[e] - a3 - w2 * h2last) * ihn;
        }
        if (sub == 0) {
            store_tile<VT, RT, ACC>(vout + i0, sv);
            store_tile<WT, RT, ACC>(w + i0, wn);
#pragma unroll
            for (int e = 0; e < RT; ++e) {
                accn += wn[e] * wn[e];
                accd += sv[e] * wn[e];
            }
        }
        accumulate_dots<JT, T, RT, VT, ACC>(raw, wn, acc);
    }
    // Partials: columns 0..nvr-1 from acc, column nvr from accd, norm slot.
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int q = 0; q < JT; ++q) {
        if (q * T < nvr) {
            ACC t = acc[q];
#pragma unroll
            for (int o = kWave / 2; o >= T; o >>= 1) t += __shfl_xor(t, o, kWave);
            const int k = sub + q * T;
            if (ln < T && k < nvr) red[wv][k] = t;
        }
    }
    {
        const ACC t = wave_sum(accd);
        if (ln == 0) red[wv][nvr] = t;
        const ACC t2 = wave_sum(accn);
        if (ln == 0) red[wv][JMAX + 1] = t2;
    }
    __syncthreads();
    const int tk = threadIdx.x;
    if (tk <= nvr || tk == JMAX + 1) {
        ACC t = red[0][tk];
#pragma unroll
        for (int q = 1; q < kWG / kWave; ++q) t += red[q][tk];
        const int slot = (tk == JMAX + 1) ? nslot : tk;
        part[(int64_t)slot * NB + blockIdx.x] = (double)t;
    }
}

// Finish the partial sums of one pass (one workgroup per slot, fixed order).
// Slots k < nv: h[k] = vscale[k] * sum (Hessenberg entries against the
// normalised v_k) and coef[k] = h[k] * vscale[k] (coefficient of stored_k).
// The norm slot: mode 1 writes ||w||^2 to ctrl->wpre2 (breakdown reference);
// mode 2 sets the storage scale sigma (sqrt(N)/||w|| for FP16 storage, else 1).
// ------------------------------- CGS2 with one reduction per step (FP64)
// Delayed re-orthogonalisation: step j >= 1 starts from q = w1_{j-1}, the
// previous step's once-projected, unnormalised vector, and u = A q (SpMV).
// One dot sweep over V_{0..j-1} takes s = V^T q (the second projection of q,
// delayed by one step), t = V^T (P u), alpha = q^T q, tau = q^T (P u) and
// ||P u||^2, and stores P u in y; one reduction; then k_dc_step finalises
// column j-1 of Hbar (h1 + s, and beta = sqrt(alpha - ||s||^2) below) and
// derives the coefficients of the update sweep, which forms the
// re-orthogonalised v_j = (q - V s) / beta and the next once-projected vector
//   w1_j = P A v_j - [V v_j] h1_j,
// with P A v_j = (P u - V_{0..j} (Hbar s)) / beta from the Arnoldi relation
// (eq. hessenberg) and h1_j from the dot products of this sweep.  Same bytes
// per step as the two-sweep variant, one reduction instead of two.
// Slots: s_l at l, t_l at nv + l (l < nv), alpha 2nv, tau 2nv + 1,
// ||P u||^2 2nv + 2.  With U = false (the cycle's last column) only s and
// alpha are taken and y is not touched.
template <int JMAX, int T, bool U>
__global__ __launch_bounds__(kWG) void k_dc_dots(int n, int64_t ldv, const double* __restrict__ V, int nv,
                                                 const double* __restrict__ q, double* __restrict__ y,
                                                 const int* __restrict__ azrp,
                                                 const int* __restrict__ azci,
                                                 const double* __restrict__ azv,
                                                 const int* __restrict__ azc2,
                                                 const double* __restrict__ azv2,
                                                 const double* __restrict__ sc, int R,
                                                 double* __restrict__ part, int NB, const Ctrl* ctrl,
                                                 int gate, int keep) {
    constexpr int JT = JMAX / T;
    constexpr int RT = 2;
    __shared__ double s_l[kMaxR];
    __shared__ double red[kWG / kWave][2 * JMAX + 3];
    if (U)
        for (int a = threadIdx.x; a < R; a += kWG) s_l[a] = sc[a];
    __syncthreads();
    if (gated(ctrl, gate)) return;
    const int sub = threadIdx.x & (T - 1);
    double as[JT], at[JT];
#pragma unroll
    for (int k = 0; k < JT; ++k) as[k] = at[k] = 0.0;
    double aa = 0.0, atau = 0.0, apu = 0.0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T) * RT;
    for (int64_t i0 = (((int64_t)blockIdx.x * kWG + threadIdx.x) / T) * RT; i0 < n; i0 += stride) {
        uint4 raw[JT];
        load_cols<JT, T, double>(V, ldv, nv, sub, i0, keep, raw);
        double qv[RT], u[RT] = {0.0, 0.0};
        load_tile<double, RT, double>(q + i0, qv);
        if (U) {
            load_tile<double, RT, double>(y + i0, u);
            if (R > 0) deflate_tile<RT, double, double>(i0, azrp, azci, azv, azc2, azv2, s_l, u);
        }
        if (sub == 0) {
            if (U) store_tile<double, RT, double>(y + i0, u);
#pragma unroll
            for (int e = 0; e < RT; ++e) {
                aa += qv[e] * qv[e];
                atau += qv[e] * u[e];
                apu += u[e] * u[e];
            }
        }
        accumulate_dots<JT, T, RT, double, double>(raw, qv, as);
        if (U) accumulate_dots<JT, T, RT, double, double>(raw, u, at);
    }
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < JT; ++k) {
        if (k * T < nv) {
            double t1 = as[k], t2 = at[k];
#pragma unroll
            for (int o = kWave / 2; o >= T; o >>= 1) {
                t1 += __shfl_xor(t1, o, kWave);
                t2 += __shfl_xor(t2, o, kWave);
            }
            const int c = sub + k * T;
            if (ln < T && c < nv) {
                red[wv][c] = t1;
                red[wv][JMAX + c] = t2;
            }
        }
    }
    {
        const double r0 = wave_sum(aa), r1 = wave_sum(atau), r2 = wave_sum(apu);
        if (ln == 0) {
            red[wv][2 * JMAX] = r0;
            red[wv][2 * JMAX + 1] = r1;
            red[wv][2 * JMAX + 2] = r2;
        }
    }
    __syncthreads();
    for (int tk = threadIdx.x; tk < 2 * JMAX + 3; tk += kWG) {
        int slot = -1;
        if (tk < nv) slot = tk;
        else if (tk >= JMAX && tk < JMAX + nv) slot = nv + (tk - JMAX);
        else if (tk >= 2 * JMAX) slot = 2 * nv + (tk - 2 * JMAX);
        if (slot < 0) continue;
        double t = red[0][tk];
#pragma unroll
        for (int w = 1; w < kWG / kWave; ++w) t += red[w][tk];
        part[(int64_t)slot * NB + blockIdx.x] = t;
    }
}

// Update sweep: qt = q - sum_l stored_l a_l (stored as column nv, times
// sigma), w = P u / beta - sum_l stored_l b_l - qt e, with lag[0] = 1/beta,
// lag[1] = e, lag[2] = sigma.  w holds q on entry (updated in place).
template <int JMAX, int T>
__global__ __launch_bounds__(kWG) void k_dc_update(int n, int64_t ldv, double* __restrict__ V, int nv,
                                                   double* __restrict__ w, const double* __restrict__ y,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ lag, const Ctrl* ctrl,
                                                   int gate, int keep) {
    constexpr int JT = JMAX / T;
    constexpr int RT = 2;
    __shared__ double a_l[JMAX], b_l[JMAX];
    const int sub = threadIdx.x & (T - 1);
    double ar[JT], br[JT];
    stage_coef<JMAX, T, double>(a, nv, a_l, sub, ar);   // synchronises
    stage_coef<JMAX, T, double>(b, nv, b_l, sub, br);
    const double ib = lag[0], ee = lag[1], sg = lag[2];
    if (gated(ctrl, gate)) return;
    double* __restrict__ vout = V + nv * ldv;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T) * RT;
    for (int64_t i0 = (((int64_t)blockIdx.x * kWG + threadIdx.x) / T) * RT; i0 < n; i0 += stride) {
        uint4 raw[JT];
        load_cols<JT, T, double>(V, ldv, nv, sub, i0, keep, raw);
        double qv[RT], u[RT], sv[RT], wn[RT];
        load_tile<double, RT, double>(w + i0, qv);
        load_tile<double, RT, double>(y + i0, u);
#pragma unroll
        for (int e = 0; e < RT; ++e) {
            const double qt = qv[e] - combine_row<JT, T, double, double>(raw, ar, e);
            sv[e] = qt * sg;
            wn[e] = u[e] * ib - combine_row<JT, T, double, double>(raw, br, e) - qt * ee;
        }
        if (sub == 0) {
            store_tile<double, RT, double>(vout + i0, sv);
            store_tile<double, RT, double>(w + i0, wn);
        }
    }
}

// Sums of the dot slots: out[b] = sum over workgroups of part[b * NB ..].
__global__ __launch_bounds__(kWG) void k_dc_sum(const double* __restrict__ part, int NB,
                                                double* __restrict__ out, const Ctrl* ctrl, int gate) {
    __shared__ double red[kWG / kWave];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int q = threadIdx.x; q < NB; q += kWG) acc += part[(int64_t)b * NB + q];
    if (gated(ctrl, gate)) return;
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[b] = acc;
}

__global__ __launch_bounds__(kWG) void k_finish(const double* __restrict__ part, int NB, int nv,
                                                int nslot, const double* __restrict__ vscale,
                                                double* __restrict__ h, double* __restrict__ coef,
                                                int mode, int half_store, double nscale,
                                                double* __restrict__ sigma, Ctrl* ctrl, int gate) {
    __shared__ double red[kWG / kWave];
    const int b = blockIdx.x;
    const int slot = (b < nv) ? b : nslot;
    // The partials are requested before the control block is tested, so the
    // two loads overlap (the test is uniform over the workgroup).
    double acc = 0;
    for (int q = threadIdx.x; q < NB; q += kWG) acc += part[(int64_t)slot * NB + q];
    const double vs = (b < nv && threadIdx.x == 0) ? vscale[b] : 0.0;
    if (gated(ctrl, gate)) return;
    acc = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    if (b < nv) {
        const double hk = vs * acc;
        h[b] = hk;
        coef[b] = hk * vs;
    } else if (mode == 1) {
        ctrl->wpre2 = acc;
    } else if (mode == 2) {
        *sigma = (half_store && acc > 0.0) ? nscale / sqrt(acc) : 1.0;
    }
}

// Givens step for column j (one wavefront).  Hbar column j is h1 + h2 with
// h_{j+1,j} = ||w||; apply the stored rotations, form the new one (rho =
// hypot(a, b), c = a/rho, s = b/rho), update g, and decide whether the cycle
// ends: |g_{j+1}| <= rtol*rho0 (eq. res), lucky breakdown
// (h_{j+1,j} <= eps * ||P A v_j||) or the iteration cap.  The column and the
// rotations are staged in LDS; one lane runs the rotation chain.
constexpr int kGT = 256;   // threads of the Givens kernel

template <bool LAG>
__global__ __launch_bounds__(kGT) void k_givens(int j, int m, const double* __restrict__ part,
                                                  int NB, int nslot, const double* __restrict__ h1,
                                                  const double* __restrict__ h2,
                                                  double* __restrict__ H, double* __restrict__ cs,
                                                  double* __restrict__ sn, double* __restrict__ g,
                                                  double* __restrict__ vscale,
                                                  const double* __restrict__ sigma,
                                                  double* __restrict__ hist, int64_t hist_cap,
                                                  double* __restrict__ Hraw, double* __restrict__ cc,
                                                  double* __restrict__ lag, Ctrl* ctrl, int gate) {
    __shared__ double col[kMaxM + 1], cl[kMaxM], sl[kMaxM], h2l[kMaxM + 1];
    __shared__ double red[kGT / kWave];
    __shared__ double ccp[LAG ? kGT : 1];
    const int tid = threadIdx.x;
    // Every independent global load is issued before the first wait: the norm
    // partials, this column's h1/h2, the stored rotations and (thread 0) the
    // scalar state.  The control-block test comes after them.
    double acc = 0;
    for (int q = tid; q < NB; q += kGT) acc += part[(int64_t)nslot * NB + q];
    double h1v = 0, h2v = 0, csv = 0, snv = 0, vsv = 0;
    if (tid <= j) {
        h1v = h1[tid];
        h2v = h2[tid];
        if (LAG) vsv = vscale[tid];
    }
    if (tid < j) {
        csv = cs[tid];
        snv = sn[tid];
    }
    double wpre2 = 0, gj = 0, target = 0, sig = 1;
    int64_t its0 = 0, maxit = 0;
    if (tid == 0) {
        wpre2 = ctrl->wpre2;
        gj = g[j];
        target = ctrl->target;
        its0 = ctrl->its;
        maxit = ctrl->max_iters;
        sig = *sigma;
    }
    if (gated(ctrl, gate)) return;
    if (tid <= j) {
        h2l[tid] = h2v;
        col[tid] = h1v + h2v;
    }
    if (tid < j) {
        cl[tid] = csv;
        sl[tid] = snv;
    }
    acc = block_sum_n<kGT>(acc, red);   // also orders the LDS writes above
    if (LAG) {
        // acc = ||w1||^2; ||w2||^2 = ||w1||^2 - ||h2||^2 (h2 against orthonormal v's).
        double q2 = 0;
        for (int i = tid; i <= j; i += kGT) q2 += h2l[i] * h2l[i];
        q2 = block_sum_n<kGT>(q2, red);
        acc = fmax(acc - q2, 0.0);
    }
    const double hn = sqrt(acc);
    if (Hraw) {
        for (int i = tid; i <= j; i += kGT) Hraw[(int64_t)i * m + j] = col[i];
        if (tid == 0) Hraw[(int64_t)(j + 1) * m + j] = hn;
    }
    if (LAG) {
        // Coefficients of the next lagged step: c_l = sum_k Hbar[l][k] h2_k over
        // the unrotated Hbar (rows l <= j, columns max(l-1,0)..j; column j is
        // col[]), times vscale[l].  Row l is split over G threads whose
        // partial sums are added in order.
        const int rows = j + 1;
        const int G = max(1, kGT / rows);
        const int l = tid % rows, grp = tid / rows;
        double v = 0;
        if (grp < G) {
            const int k0 = (l > 0 ? l - 1 : 0), k1 = j;   // band columns < j
            const int span = (k1 - k0 + G - 1) / G;
            const int a0 = k0 + grp * span, a1 = min(k1, a0 + span);
            for (int k = a0; k < a1; ++k) v += Hraw[(int64_t)l * m + k] * h2l[k];
        }
        ccp[tid] = v;
        __syncthreads();
        if (tid < rows) {
            double c = ccp[tid];
            for (int q = 1; q < G; ++q) c += ccp[q * rows + tid];
            c += col[tid] * h2l[j];
            cc[tid] = c * vsv;
        }
    }
    if (tid != 0) return;
    const double wpre = sqrt(wpre2);
    // The lagged norm comes from a difference of squares: its rounding error is
    // about sqrt(eps) * ||w1||, so a breakdown is declared below that level.
    const double bd_tol = LAG ? 1.4901161193847656e-08 : 2.220446049250313e-16;
    const int bd = !(hn > bd_tol * wpre);
    double a = col[0];
#pragma unroll 8
    for (int i = 0; i < j; ++i) {
        const double c = cl[i], sv = sl[i], bb = col[i + 1];
        H[(int64_t)i * m + j] = c * a + sv * bb;
        a = -sv * a + c * bb;
    }
    double rho = hypot(a, hn);
    double cj, sj;
    if (hn == 0.0) {
        cj = 1.0;
        sj = 0.0;
        rho = a;
    } else {
        cj = a / rho;
        sj = hn / rho;
    }
    cs[j] = cj;
    sn[j] = sj;
    H[(int64_t)j * m + j] = rho;
    H[(int64_t)(j + 1) * m + j] = 0.0;
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
    vscale[j + 1] = bd ? 0.0 : 1.0 / (sig * hn);
    if (LAG) {
        lag[0] = h2l[j];
        lag[1] = bd ? 0.0 : 1.0 / hn;
        lag[2] = sig;
    }
    const int64_t its = its0 + 1;
    ctrl->its = its;
    if (hist && ctrl->hist_base + its - 1 < hist_cap) hist[ctrl->hist_base + its - 1] = fabs(sj * gj);
    ctrl->k = j + 1;
    ctrl->breakdown = bd;
    const bool est = fabs(sj * gj) <= target;
    if (est) ctrl->est_conv = 1;
    if (est || bd || its >= maxit) ctrl->stop = 1;
}

// Back substitution R_k y = g_{1:k} (column-oriented, R staged in LDS);
// coef[i] = y_i * vscale[i] (coefficient of stored_i in x_hat += V_k y).
// Single-reduction CGS2: column j-1 of Hbar from the slot sums dcs of
// k_dc_dots (nv = j): s_l = vscale_l dcs[l], t_l = vscale_l dcs[j + l],
// alpha, tau, ||P u||^2; beta = sqrt(alpha - ||s||^2) (Pythagoras: v_l
// orthonormal), column = h1 + s over rows < j and beta at row j; Givens as in
// k_givens.  Unless FINAL, the coefficients of the update sweep: c = Hbar s
// (unrotated Hbar, band rows), h1 of column j (l < j: (t_l - c_l)/beta;
// l = j: ((tau - s.t)/beta - c_j)/beta), d = c/beta + h1, ca = s vscale,
// cb = d vscale (l < j), lag = {1/beta, d_j/beta, sigma}, and ||P A v_j||^2
// for the next breakdown test.  h1 holds column j-1's first-projection
// coefficients on entry and column j's on exit.
template <bool FINAL>
__global__ __launch_bounds__(kGT) void k_dc_step(int j, int m, const double* __restrict__ dcs,
                                                 double* __restrict__ h1, double* __restrict__ H,
                                                 double* __restrict__ cs, double* __restrict__ sn,
                                                 double* __restrict__ g, double* __restrict__ vscale,
                                                 const double* __restrict__ sigma,
                                                 double* __restrict__ hist, int64_t hist_cap,
                                                 double* __restrict__ Hraw, double* __restrict__ ca,
                                                 double* __restrict__ cb, double* __restrict__ lag,
                                                 Ctrl* ctrl, int gate) {
    __shared__ double sl[kMaxM + 1], tl[kMaxM + 1], col[kMaxM + 1], cl[kMaxM], snl[kMaxM];
    __shared__ double cc[kMaxM + 1], vsl[kMaxM + 1];
    __shared__ double red[kGT / kWave];
    const int tid = threadIdx.x;
    const int jc = j - 1;
    double sv = 0.0, tv = 0.0, h1v = 0.0, vsv = 0.0, csv = 0.0, snv = 0.0;
    if (tid < j) {
        vsv = vscale[tid];
        sv = dcs[tid];
        if (!FINAL) tv = dcs[j + tid];
        h1v = h1[tid];
    }
    if (tid < jc) {
        csv = cs[tid];
        snv = sn[tid];
    }
    double alpha = 0.0, tau = 0.0, pu2 = 0.0, wpre2 = 0.0, gj = 0.0, target = 0.0, sig = 1.0;
    int64_t its0 = 0, maxit = 0;
    if (tid == 0) {
        alpha = dcs[2 * j];
        if (!FINAL) {
            tau = dcs[2 * j + 1];
            pu2 = dcs[2 * j + 2];
        }
        wpre2 = ctrl->wpre2;
        gj = g[jc];
        target = ctrl->target;
        its0 = ctrl->its;
        maxit = ctrl->max_iters;
        sig = *sigma;
    }
    if (gated(ctrl, gate)) return;
    sv *= vsv;
    tv *= vsv;
    if (tid < j) {
        sl[tid] = sv;
        tl[tid] = tv;
        col[tid] = h1v + sv;
        vsl[tid] = vsv;
    }
    if (tid < jc) {
        cl[tid] = csv;
        snl[tid] = snv;
    }
    double ss = block_sum_n<kGT>(sv * sv, red);   // also orders the LDS writes above
    double st = block_sum_n<kGT>(sv * tv, red);
    double beta = 0.0;
    if (tid == 0) {
        beta = sqrt(fmax(alpha - ss, 0.0));
        col[j] = beta;
    }
    __syncthreads();
    beta = col[j];
    for (int i = tid; i <= j; i += kGT) Hraw[(int64_t)i * m + jc] = col[i];
    // sqrt(eps) * ||P A v_{j-1}||: the Pythagorean norm carries about sqrt(eps)
    // of relative rounding error.
    const int bd = !(beta > 1.4901161193847656e-08 * sqrt(tid == 0 ? wpre2 : 0.0)) ? 1 : 0;
    __syncthreads();
    double ib = 0.0;
    if (!FINAL) {
        // c = Hbar(0:j, 0:j-1) s over the band (row i: columns i-1 .. j-1).
        // Columns < j-1 from Hraw, column j-1 from LDS (just formed).
        double c = 0.0;
        if (tid <= j) {
            for (int l = (tid > 0 ? tid - 1 : 0); l < jc; ++l) c += Hraw[(int64_t)tid * m + l] * sl[l];
            c += col[tid] * sl[jc];
        }
        if (tid <= j) cc[tid] = c;
        __syncthreads();
        ib = beta > 0.0 ? 1.0 / beta : 0.0;
        const double vjpu = (tau - st) * ib;   // thread 0 only (tau, st valid there)
        if (tid < j) {
            const double h1n = (tl[tid] - cc[tid]) * ib;
            const double d = cc[tid] * ib + h1n;
            ca[tid] = sl[tid] * vsl[tid];
            cb[tid] = d * vsl[tid];
            h1[tid] = h1n;
        }
        double ct = block_sum_n<kGT>(tid < j ? cc[tid] * tl[tid] : 0.0, red);
        double c2 = block_sum_n<kGT>(tid <= j ? cc[tid] * cc[tid] : 0.0, red);
        if (tid == 0) {
            const double h1j = (vjpu - cc[j]) * ib;
            const double dj = cc[j] * ib + h1j;
            h1[j] = h1j;
            lag[0] = bd ? 0.0 : ib;
            lag[1] = bd ? 0.0 : dj * ib;
            lag[2] = sig;
            const double z2 = (pu2 - 2.0 * (ct + cc[j] * vjpu) + c2) * ib * ib;
            ctrl->wpre2 = fmax(z2, 0.0);
        }
    }
    if (tid != 0) return;
    double a = col[0];
    for (int i = 0; i < jc; ++i) {
        const double c = cl[i], sv2 = snl[i], bb = col[i + 1];
        H[(int64_t)i * m + jc] = c * a + sv2 * bb;
        a = -sv2 * a + c * bb;
    }
    double rho = hypot(a, beta);
    double cj, sj;
    if (beta == 0.0) {
        cj = 1.0;
        sj = 0.0;
        rho = a;
    } else {
        cj = a / rho;
        sj = beta / rho;
    }
    cs[jc] = cj;
    sn[jc] = sj;
    H[(int64_t)jc * m + jc] = rho;
    H[(int64_t)j * m + jc] = 0.0;
    g[j] = -sj * gj;
    g[jc] = cj * gj;
    vscale[j] = bd ? 0.0 : 1.0 / (sig * beta);
    const int64_t its = its0 + 1;
    ctrl->its = its;
    if (hist && ctrl->hist_base + its - 1 < hist_cap) hist[ctrl->hist_base + its - 1] = fabs(sj * gj);
    ctrl->k = j;
    ctrl->breakdown = bd;
    const bool est = fabs(sj * gj) <= target;
    if (est) ctrl->est_conv = 1;
    if (est || bd || its >= maxit || FINAL) ctrl->stop = 1;
}

__global__ __launch_bounds__(kWG) void k_backsolve(int m, const double* __restrict__ H,
                                                   const double* __restrict__ g,
                                                   const double* __restrict__ vscale,
                                                   double* __restrict__ coef, int* cyc_k,
                                                   int cyc_cap, Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ double Rl[kMaxM * kMaxM];
    __shared__ double gl[kMaxM], yl[kMaxM];
    const int k = ctrl->k;
    if (threadIdx.x == 0 && cyc_k && ctrl->cycles - 1 < cyc_cap) cyc_k[ctrl->cycles - 1] = k;
    for (int q = threadIdx.x; q < k * k; q += kWG) {
        const int i = q / k, c = q % k;
        Rl[q] = (c >= i) ? H[(int64_t)i * m + c] : 0.0;
    }
    for (int i = threadIdx.x; i < k; i += kWG) gl[i] = g[i];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        const double yi = gl[i] / Rl[i * k + i];
        for (int l = threadIdx.x; l < i; l += kWG) gl[l] -= Rl[l * k + i] * yi;
        if (threadIdx.x == 0) yl[i] = yi;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < k; i += kWG) coef[i] = yl[i] * vscale[i];
}

// x_hat += sum_{t < k} stored_t * coef[t]  (eq. new_sol); k from the control block.
template <typename VT>
__global__ __launch_bounds__(kWG) void k_xupdate(int n, int64_t ldv, const VT* __restrict__ V,
                                                 const double* __restrict__ coef,
                                                 double* __restrict__ xh, Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ double c_l[kMaxM];
    const int k = ctrl->k;
    for (int t = threadIdx.x; t < k; t += kWG) c_l[t] = coef[t];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        double acc = 0;
        int t = 0;
        for (; t + 4 <= k; t += 4) {
            const double a0 = (double)ld_f(V + t * ldv + i);
            const double a1 = (double)ld_f(V + (t + 1) * ldv + i);
            const double a2 = (double)ld_f(V + (t + 2) * ldv + i);
            const double a3 = (double)ld_f(V + (t + 3) * ldv + i);
            acc += a0 * c_l[t];
            acc += a1 * c_l[t + 1];
            acc += a2 * c_l[t + 2];
            acc += a3 * c_l[t + 3];
        }
        for (; t < k; ++t) acc += (double)ld_f(V + t * ldv + i) * c_l[t];
        xh[i] += acc;
    }
}

// rho0 = ||r0|| (or the caller's override), target = rtol * rho0.
__global__ void k_init(const double* __restrict__ part, int NB, int nslot, double rtol,
                       double r0_override, Ctrl* ctrl) {
    __shared__ double red[kWG / kWave];
    double acc = 0;
    for (int q = threadIdx.x; q < NB; q += kWG) acc += part[(int64_t)nslot * NB + q];
    acc = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    const double rho0 = r0_override > 0.0 ? r0_override : sqrt(acc);
    ctrl->rho0 = rho0;
    ctrl->target = rtol * rho0;
    if (!isfinite(acc) || !isfinite(rho0)) {
        ctrl->done = 1;
        ctrl->status = kStatusNonFinite;
    } else if (rho0 == 0.0) {
        ctrl->done = 1;
        ctrl->status = kStatusOk;
    }
}

// Restart decision from beta = ||P r||: converged, cap reached, or start a
// new cycle with g = beta e1 and v_1 = p / beta.
__global__ void k_decide(const double* __restrict__ part, int NB, int nslot, int m,
                         int half_store, double nscale, double* __restrict__ g,
                         double* __restrict__ vscale, double* __restrict__ sigma0, int trust_est,
                         Ctrl* ctrl) {
    __shared__ double red[kWG / kWave];
    if (ctrl->done) return;
    double acc = 0;
    for (int q = threadIdx.x; q < NB; q += kWG) acc += part[(int64_t)nslot * NB + q];
    acc = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(acc);
    ctrl->beta = beta;
    if (!isfinite(beta)) {
        ctrl->done = 1;
        ctrl->status = kStatusNonFinite;
    } else if (beta <= ctrl->target || (trust_est && ctrl->est_conv)) {
        ctrl->done = 1;
        ctrl->status = kStatusOk;
    } else if (ctrl->its >= ctrl->max_iters) {
        ctrl->done = 1;
        ctrl->status = kStatusMaxIter;
    } else {
        ctrl->stop = 0;
        ctrl->k = 0;
        ctrl->cycles += 1;
        g[0] = beta;
        for (int i = 1; i <= m; ++i) g[i] = 0.0;
        const double sg = half_store ? nscale / beta : 1.0;
        *sigma0 = sg;
        vscale[0] = 1.0 / (sg * beta);
    }
}

// V[:,0] = sigma0 * p.
template <typename VT, typename WT>
__global__ __launch_bounds__(kWG) void k_store_v0(int n, const WT* __restrict__ p,
                                                  const double* __restrict__ sigma0,
                                                  VT* __restrict__ v0, const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    const double sg = *sigma0;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride)
        st_v(v0 + i, (decltype(ld_f(v0)))((double)p[i] * sg));
}

// x = x_hat + Z s  (final coarse correction; s = E^{-1} Z^T (b - A x_hat)).
__global__ __launch_bounds__(kWG) void k_correct(int n, const int* __restrict__ zrp,
                                                 const int* __restrict__ zci,
                                                 const double* __restrict__ zv,
                                                 const double* __restrict__ s, int R,
                                                 const double* __restrict__ xh,
                                                 double* __restrict__ x) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        double v = xh[i];
        if (R > 0)
            for (int q = zrp[i]; q < zrp[i + 1]; ++q) v += zv[q] * s[zci[q]];
        x[i] = v;
    }
}

// Sum NB partials of one slot into *out (one workgroup, fixed order).
__global__ void k_sum_slot(const double* __restrict__ part, int NB, int nslot,
                           double* __restrict__ out) {
    __shared__ double red[kWG / kWave];
    double acc = 0;
    for (int q = threadIdx.x; q < NB; q += kWG) acc += part[(int64_t)nslot * NB + q];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) *out = acc;
}

// Mixed precision: rhat = (b - A x) / ||b - A x|| in FP32, from the FP64
// residual r and its squared norm.
__global__ __launch_bounds__(kWG) void k_scale_to_f32(int n, const double* __restrict__ r,
                                                      const double* __restrict__ nrm2,
                                                      float* __restrict__ out) {
    const double inv = 1.0 / sqrt(*nrm2);
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride)
        out[i] = (float)(r[i] * inv);
}

// Mixed precision: x += alpha * d with alpha = ||r|| (FP64).
__global__ __launch_bounds__(kWG) void k_axpy_norm(int n, const double* __restrict__ nrm2,
                                                   const double* __restrict__ d,
                                                   double* __restrict__ x) {
    const double a = sqrt(*nrm2);
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) x[i] += a * d[i];
}

__global__ void k_ctrl_reset(Ctrl* ctrl, int64_t max_iters, int64_t hist_base) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctrl c = {};
        c.max_iters = max_iters;
        c.hist_base = hist_base;
        c.stop = 1;
        *ctrl = c;
    }
}

__global__ __launch_bounds__(kWG) void k_fill(double* __restrict__ p, int64_t n, double v) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(kWG) void k_copy_f64(const double* __restrict__ a, double* __restrict__ b,
                                                  int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// ====================================================================== host
// Launch helpers used by the solve engine.  All launches go to `st`.

// Per-kernel timing: arm_kernel_events() hands a pair of timing events to the
// next kernel enqueued through launch() on this thread; that launch records
// the kernel's own start and end timestamps in them (hipExtLaunchKernel), so
// the elapsed time covers the kernel alone, as a kernel trace reports it.
static thread_local hipEvent_t t_ev_start = nullptr;
static thread_local hipEvent_t t_ev_stop = nullptr;

void arm_kernel_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}

bool disarm_kernel_events() {
    const bool pending = t_ev_start != nullptr;
    t_ev_start = t_ev_stop = nullptr;
    return pending;
}

bool take_kernel_events(hipEvent_t* start, hipEvent_t* stop) {
    if (!t_ev_start) return false;
    *start = t_ev_start;
    *stop = t_ev_stop;
    t_ev_start = t_ev_stop = nullptr;
    return true;
}

// Workgroups of one streaming pass: as many as the device holds at once
// (a single round, so every workgroup gets the same share of rows), at most
// cap.  Queried once per kernel and device.
static int resident_grid(const void* k, int cap) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int g = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({dev, k});
        if (it != cache.end()) {
            g = it->second;
        } else {
            int per_cu = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kWG, 0) != hipSuccess ||
                per_cu < 1)
                per_cu = 1;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                    hipSuccess ||
                cus < 1)
                cus = 1;
            g = per_cu * cus;
            cache[{dev, k}] = g;
        }
    }
    return std::max(1, std::min(g, cap));
}

template <typename... KA, typename... A>
static inline void launch(void (*k)(KA...), dim3 g, dim3 b, uint32_t sh, hipStream_t st,
                          A... args) {
    if (t_ev_start) {
        hipEvent_t e0 = t_ev_start, e1 = t_ev_stop;
        t_ev_start = t_ev_stop = nullptr;
        hipExtLaunchKernelGGL(k, g, b, sh, st, e0, e1, 0u, static_cast<KA>(args)...);
    } else {
        k<<<g, b, sh, st>>>(static_cast<KA>(args)...);
    }
}

template <typename AT, typename XT, typename YT, typename ACC>
static void spmv_dispatch(int L, int NB, hipStream_t st, int n, const int* rp, const int* ci,
                          const AT* v, const XT* x, const double* scale, YT* y, const Ctrl* c,
                          int gate) {
    dim3 g(NB), b(kWG);
    if (L == -256) {
        launch(k_spmv_stream<256, 0, false, AT, XT, double, YT, ACC>, g, 256, 0, st, n, rp, ci, v, x, scale, nullptr, y, nullptr, 0, NB, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c, gate);
        return;
    }
    if (L <= 0) {
        launch(k_spmv_stream<128, 0, false, AT, XT, double, YT, ACC>, g, 128, 0, st, n, rp, ci, v, x, scale, nullptr, y, nullptr, 0, NB, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c, gate);
        return;
    }
    switch (L) {
        case 1: launch(k_spmv<1, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
        case 2: launch(k_spmv<2, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
        case 4: launch(k_spmv<4, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
        case 8: launch(k_spmv<8, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
        case 16: launch(k_spmv<16, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
        case 32: launch(k_spmv<32, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
        default: launch(k_spmv<64, AT, XT, YT, ACC>, g, b, 0, st, n, rp, ci, v, x, scale, y, c, gate); break;
    }
}

template <typename AT, typename BT, typename RT, typename ACC>
static void residual_dispatch(int L, int NB, hipStream_t st, int n, const int* rp, const int* ci,
                              const AT* v, const double* x, const BT* b, RT* r, double* part,
                              int slot, const Ctrl* c, int gate) {
    dim3 g(NB), bl(kWG);
    if (L == -256) {
        k_spmv_stream<256, 1, false, AT, double, BT, RT, ACC><<<g, 256, 0, st>>>(n, rp, ci, v, x, nullptr, b, r, part, slot, NB, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c, gate);
        return;
    }
    if (L <= 0) {
        k_spmv_stream<128, 1, false, AT, double, BT, RT, ACC><<<g, 128, 0, st>>>(n, rp, ci, v, x, nullptr, b, r, part, slot, NB, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c, gate);
        return;
    }
    switch (L) {
        case 1: k_residual<1, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
        case 2: k_residual<2, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
        case 4: k_residual<4, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
        case 8: k_residual<8, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
        case 16: k_residual<16, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
        case 32: k_residual<32, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
        default: k_residual<64, AT, BT, RT, ACC><<<g, bl, 0, st>>>(n, rp, ci, v, x, b, r, part, slot, NB, c, gate); break;
    }
}

// Stream SpMV (MODE 0) or residual (MODE 1) with the fused Z^T partials.
template <int MODE, typename AT, typename XT, typename BT, typename YT, typename ACC>
static void stream_fused(const EngineArgs& e, const AT* vals, const XT* x, const double* scale,
                         const BT* b, YT* y, int slot, int gate) {
    if (e.fuse_rb == 256)
        launch(k_spmv_stream<256, MODE, true, AT, XT, BT, YT, ACC>, e.NB, 256, 0, e.st, 
            e.n, e.rowptr, e.colind, vals, x, scale, b, y, e.part, slot, e.NB, e.zrp, e.zci, e.zv,
            e.bb_ptr, e.bb_col, e.slot_pos, e.zc1, e.zv1, e.tpart, e.ctrl, gate);
    else
        launch(k_spmv_stream<128, MODE, true, AT, XT, BT, YT, ACC>, e.NB, 128, 0, e.st, 
            e.n, e.rowptr, e.colind, vals, x, scale, b, y, e.part, slot, e.NB, e.zrp, e.zci, e.zv,
            e.bb_ptr, e.bb_col, e.slot_pos, e.zc1, e.zv1, e.tpart, e.ctrl, gate);
}

template <int MODE, int WMAX, typename AT, typename XT, typename BT, typename YT, typename ACC>
static void sell_launch_w(const EngineArgs& e, const XT* x, const double* scale, const BT* b, YT* y,
                          int slot, int gate) {
    const AT* sv = reinterpret_cast<const AT*>(e.sell_val);
    // MODE 0 needs no per-block partials: one block per 256-row block.  MODE 1
    // writes one norm partial per block, so it keeps the NB-block grid.
    const int64_t n = e.n;
    if (e.R > 0 && e.fuse_rb == 256) {
        const int grid = MODE == 0 ? (int)std::max<int64_t>(1, (n + kWG - 1) / kWG) : e.NB;
        launch(k_spmv_sell<MODE, true, WMAX, kWG, AT, XT, BT, YT, ACC>, grid, kWG, 0, e.st,
            e.n, e.sell_off, e.sell_perm, e.sell_wuni, e.sell_col, sv, x, scale, b, y, e.part, slot, e.NB, e.zrp, e.zci, e.zv,
            e.bb_ptr, e.bb_col, e.slot_pos, e.zc1, e.zv1, e.tpart, e.ctrl, gate);
    } else {
        const int grid = MODE == 0 ? (int)std::max<int64_t>(1, (n + kWG - 1) / kWG) : e.NB;
        launch(k_spmv_sell<MODE, false, WMAX, kWG, AT, XT, BT, YT, ACC>, grid, kWG, 0, e.st,
            e.n, e.sell_off, e.sell_perm, e.sell_wuni, e.sell_col, sv, x, scale, b, y, e.part, slot, e.NB, nullptr, nullptr,
            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, e.ctrl, gate);
    }
}

template <int MODE, typename AT, typename XT, typename BT, typename YT, typename ACC>
static void sell_launch(const EngineArgs& e, const XT* x, const double* scale, const BT* b, YT* y,
                        int slot, int gate) {
    // Fully unrolled rows up to 25 entries (the smallest instance that holds
    // the longest row), chunked rows beyond (streamed when the matrix does not
    // fit in the last-level cache).
    if (e.sell_stream && e.sell_wmax <= 9)
        sell_launch_w<MODE, kSellStreamW + 9, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
    else if (e.sell_wmax <= 9) sell_launch_w<MODE, 9, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
    else if (e.sell_wmax <= 12) sell_launch_w<MODE, 12, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
    else if (e.sell_wmax <= 16) sell_launch_w<MODE, 16, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
    else if (e.sell_wmax <= 25) sell_launch_w<MODE, 25, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
    else if (e.sell_stream) sell_launch_w<MODE, -1, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
    else sell_launch_w<MODE, 0, AT, XT, BT, YT, ACC>(e, x, scale, b, y, slot, gate);
}

static int jmax_for(int nv) {
    if (nv <= 8) return 8;
    if (nv <= 16) return 16;
    if (nv <= 24) return 24;
    if (nv <= 32) return 32;
    if (nv <= 40) return 40;
    if (nv <= 48) return 48;
    if (nv <= 56) return 56;
    if (nv <= 64) return 64;
    if (nv <= 80) return 80;
    return 96;
}

// Lanes per tile of the pass kernels: at most 16 basis tiles (64 VGPRs) per
// lane, so no instantiation spills.
template <int J, typename VT>
struct LanesFor {
    static constexpr int base = J <= 16 ? 1 : (J <= 32 ? 2 : (J <= 64 ? 4 : 8));
    // A 16-byte FP16 tile holds 8 rows: halve the columns per lane.
    static constexpr int value = sizeof(VT) == 2 ? 2 * base : base;
};

// The two-sweep first pass keeps two coefficient sets per lane: FP32/FP64
// bases spread the columns over twice as many lanes to stay at >= 4 waves
// per SIMD (FP16 tiles are already spread), except FP64 bases of 33..64
// columns, where 4 lanes (10-16 columns each, 3-4 waves per SIMD) measured
// faster than 8.
template <int J, typename VT>
struct LanesForLag {
    static constexpr int spread = 2 * LanesFor<J, VT>::value > 16 ? 16 : 2 * LanesFor<J, VT>::value;
    static constexpr int value = sizeof(VT) == 2 ? LanesFor<J, VT>::value
                                 : (sizeof(VT) == 8 && J > 32 && J <= 64 ? 4 : spread);
};

#define GM_JMAX_CASE(JV, VTT, CALL) \
    case JV: { constexpr int J = JV; constexpr int T = LanesFor<J, VTT>::value; CALL; } break;
#define GM_JMAX_SWITCH(nv, VTT, CALL)   \
    switch (jmax_for(nv)) {             \
        GM_JMAX_CASE(8, VTT, CALL)      \
        GM_JMAX_CASE(16, VTT, CALL)     \
        GM_JMAX_CASE(24, VTT, CALL)     \
        GM_JMAX_CASE(32, VTT, CALL)     \
        GM_JMAX_CASE(40, VTT, CALL)     \
        GM_JMAX_CASE(48, VTT, CALL)     \
        GM_JMAX_CASE(56, VTT, CALL)     \
        GM_JMAX_CASE(64, VTT, CALL)     \
        GM_JMAX_CASE(80, VTT, CALL)     \
        default: { constexpr int J = 96; constexpr int T = LanesFor<J, VTT>::value; CALL; } break; \
    }

// ---------------------------------------------------------------- engine
// Enqueues the kernels of a solve for one operator (A or A^T) in one
// precision.  AT: matrix values, VT: basis storage, WT: work vectors,
// ACC: accumulation type.
template <typename AT, typename VT, typename WT, typename ACC>
struct Engine {
    const EngineArgs& e;
    explicit Engine(const EngineArgs& a) : e(a) {}

    VT* V() const { return reinterpret_cast<VT*>(e.V); }
    VT* Vcol(int k) const { return V() + (int64_t)k * e.ldv; }
    WT* y() const { return reinterpret_cast<WT*>(e.y); }
    WT* w() const { return reinterpret_cast<WT*>(e.w); }
    WT* p() const { return reinterpret_cast<WT*>(e.p); }
    WT* r() const { return reinterpret_cast<WT*>(e.r); }
    const AT* vals() const { return reinterpret_cast<const AT*>(e.vals); }
    const AT* azv() const { return reinterpret_cast<const AT*>(e.azv); }
    const AT* azv1() const { return reinterpret_cast<const AT*>(e.azv1); }
    static constexpr int kHalf = std::is_same<VT, __half>::value ? 1 : 0;

    bool fused() const { return e.R > 0 && e.fuse_rb != 0; }

    // Grid of an Arnoldi pass: one full round of resident workgroups, or the
    // plan's fixed grid when pass_grid is 0.
    int grid_for(const void* k) const {
        return e.pass_grid ? resident_grid(k, e.nbcap) : e.NB;
    }

    void coarse_slots(double* s, int gate) const {
        k_coarse_slots<<<1, kCT, 0, e.st>>>(e.R, e.ab_ptr, e.tpart, e.Einv, e.trans, s, e.ctrl,
                                            gate);
    }

    void coarse(const WT* vec, double* s, int gate) const {
        if (e.R == 0) return;
        k_zt<WT><<<e.R * e.MC, kWG, 0, e.st>>>(e.R, e.MC, e.CH, e.ztrp, e.ztci, e.ztv, vec, e.tpart,
                                              e.ctrl, gate);
        k_coarse<<<1, kCT, 0, e.st>>>(e.R, e.MC, e.tpart, e.Einv, e.trans, s, e.ctrl, gate);
    }

    // Residual of x_hat, its deflated version p = P r into e.p, and the
    // restart decision (or the initialisation when `init`).
    template <typename BT>
    void restart_block(const BT* b, bool init, double rtol, double r0_override) const {
        if (e.L == kSell) {
            sell_launch<1, AT, double, BT, WT, ACC>(e, e.xh, nullptr, b, r(), e.nslot, init ? 0 : 1);
            if (init) k_init<<<1, kWG, 0, e.st>>>(e.part, e.NB, e.nslot, rtol, r0_override, e.ctrl);
            if (fused()) coarse_slots(e.s_res, init ? 0 : 1);
            else coarse(r(), e.s_res, init ? 0 : 1);
        } else if (fused()) {
            stream_fused<1, AT, double, BT, WT, ACC>(e, vals(), e.xh, nullptr, b, r(), e.nslot,
                                                      init ? 0 : 1);
            if (init) k_init<<<1, kWG, 0, e.st>>>(e.part, e.NB, e.nslot, rtol, r0_override, e.ctrl);
            coarse_slots(e.s_res, init ? 0 : 1);
        } else {
            residual_dispatch<AT, BT, WT, ACC>(e.L, e.NB, e.st, e.n, e.rowptr, e.colind, vals(), e.xh,
                                               b, r(), e.part, e.nslot, e.ctrl, init ? 0 : 1);
            if (init) k_init<<<1, kWG, 0, e.st>>>(e.part, e.NB, e.nslot, rtol, r0_override, e.ctrl);
            coarse(r(), e.s_res, init ? 0 : 1);
        }
        k_pass1<8, 1, VT, WT, AT, ACC><<<e.NB, kWG, 0, e.st>>>(e.n, e.ldv, V(), 0, r(), e.azrp, e.azci,
                                                            azv(), e.azc1, azv1(), e.s_res, e.R, p(), e.part,
                                                            e.nslot, e.NB, e.ctrl, 1, e.cache_cols);
        k_decide<<<1, kWG, 0, e.st>>>(e.part, e.NB, e.nslot, e.m, kHalf, e.nscale, e.g, e.vscale,
                                      e.sigma0, e.trust_est, e.ctrl);
        k_store_v0<VT, WT><<<e.NB, kWG, 0, e.st>>>(e.n, p(), e.sigma0, Vcol(0), e.ctrl, 1);
    }

    // Adaptive deflation (FP64 only): s = C U^T x before the SpMV of input x,
    // y += (A U) s after it, so y = A M^{-1} x.
    void op_pre(const VT* x, const double* scale) const {
        if constexpr (std::is_same<VT, double>::value)
            if (e.adapt) adapt_pre(e, x, scale);
    }
    void op_pre_w(const WT* x) const {
        if constexpr (std::is_same<WT, double>::value)
            if (e.adapt) adapt_pre(e, x, nullptr);
    }
    void op_post() const {
        if constexpr (std::is_same<WT, double>::value)
            if (e.adapt) adapt_post(e, y());
    }

    void step(int j) const {
        const int nv = j + 1;
        op_pre(Vcol(j), e.vscale + j);
        if (e.timer) e.timer->begin(0, j);
        if (e.L == kSell)
            sell_launch<0, AT, VT, double, WT, ACC>(e, Vcol(j), e.vscale + j, nullptr, y(), 0, 2);
        else if (fused())
            stream_fused<0, AT, VT, double, WT, ACC>(e, vals(), Vcol(j), e.vscale + j, nullptr, y(),
                                                      0, 2);
        else
            spmv_dispatch<AT, VT, WT, ACC>(e.L, e.NB, e.st, e.n, e.rowptr, e.colind, vals(), Vcol(j),
                                           e.vscale + j, y(), e.ctrl, 2);
        if (e.timer) e.timer->end(0, j);
        op_post();
        if (fused()) coarse_slots(e.s_step, 2);
        else coarse(y(), e.s_step, 2);
        if (e.timer) e.timer->begin(1, j);
        int g1 = 0, g2 = 0, g3 = 0;
        GM_JMAX_SWITCH(nv, VT, ({
            auto kf = k_pass1<J, T, VT, WT, AT, ACC>;
            g1 = grid_for((const void*)kf);
            launch(kf, g1, kWG, 0, e.st, e.n, e.ldv, V(), nv, y(), e.azrp, e.azci, azv(), e.azc1,
                   azv1(), e.s_step, e.R, w(), e.part, e.nslot, g1, e.ctrl, 2, e.cache_cols);
        }));
        if (e.timer) e.timer->end(1, j);
        k_finish<<<nv + 1, kWG, 0, e.st>>>(e.part, g1, nv, e.nslot, e.vscale, e.h1, e.coef1, 1,
                                           kHalf, e.nscale, e.sigma, e.ctrl, 2);
        if (e.timer) e.timer->begin(2, j);
        GM_JMAX_SWITCH(nv, VT, ({
            auto kf = k_pass2<J, T, VT, WT, ACC>;
            g2 = grid_for((const void*)kf);
            launch(kf, g2, kWG, 0, e.st, e.n, e.ldv, V(), nv, w(), e.coef1, e.part, e.nslot, g2,
                   e.ctrl, 2, e.cache_cols);
        }));
        if (e.timer) e.timer->end(2, j);
        k_finish<<<nv + 1, kWG, 0, e.st>>>(e.part, g2, nv, e.nslot, e.vscale, e.h2, e.coef2, 2,
                                           kHalf, e.nscale, e.sigma, e.ctrl, 2);
        if (e.timer) e.timer->begin(3, j);
        GM_JMAX_SWITCH(nv, VT, ({
            auto kf = k_pass3<J, T, VT, WT, ACC>;
            g3 = grid_for((const void*)kf);
            launch(kf, g3, kWG, 0, e.st, e.n, e.ldv, V(), nv, w(), e.coef2, e.sigma, e.part,
                   e.nslot, g3, e.ctrl, 2, e.cache_cols);
        }));
        if (e.timer) e.timer->end(3, j);
        launch(k_givens<false>, 1, kGT, 0, e.st, j, e.m, e.part, g3, e.nslot, e.h1, e.h2, e.H, e.cs,
               e.sn, e.g, e.vscale, e.sigma, e.hist, e.hist_cap, e.Hraw, nullptr, nullptr, e.ctrl,
               2);
    }

    // Step j of the two-pass variant (see k_pass1_lag).
    void step_lag(int j) const {
        const int nv = j + 1;
        if (j == 0) op_pre(Vcol(0), e.vscale);
        else op_pre_w(w());
        if (e.timer) e.timer->begin(0, j);
        if (j == 0) {
            spmv_any<VT>(Vcol(0), e.vscale);
        } else {
            spmv_any<WT>(w(), nullptr);
        }
        if (e.timer) e.timer->end(0, j);
        op_post();
        if (fused()) coarse_slots(e.s_step, 2);
        else coarse(y(), e.s_step, 2);
        if (e.timer) e.timer->begin(1, j);
        int g1 = 0, g2 = 0;
        if (j == 0) {
            auto kf = k_pass1<8, 1, VT, WT, AT, ACC>;
            g1 = grid_for((const void*)kf);
            launch(kf, g1, kWG, 0, e.st, e.n, e.ldv, V(), 1, y(), e.azrp, e.azci, azv(), e.azc1,
                   azv1(), e.s_step, e.R, w(), e.part, e.nslot, g1, e.ctrl, 2, e.cache_cols);
        } else {
            GM_JMAX_SWITCH(j, VT, ({
                auto kf = k_pass1_lag<J, LanesForLag<J, VT>::value, VT, WT, AT, ACC>;
                g1 = grid_for((const void*)kf);
                launch(kf, g1, kWG, 0, e.st, e.n, e.ldv, V(), j, w(), y(), e.azrp, e.azci, azv(),
                       e.azc1, azv1(), e.s_step, e.R, e.coef2, e.cc, e.lag, e.part, e.nslot, g1,
                       e.ctrl, 2, e.cache_cols);
            }));
        }
        if (e.timer) e.timer->end(1, j);
        k_finish<<<nv + 1, kWG, 0, e.st>>>(e.part, g1, nv, e.nslot, e.vscale, e.h1, e.coef1, 1,
                                           kHalf, e.nscale, e.sigma, e.ctrl, 2);
        if (e.timer) e.timer->begin(2, j);
        GM_JMAX_SWITCH(nv, VT, ({
            auto kf = k_pass2<J, T, VT, WT, ACC>;
            g2 = grid_for((const void*)kf);
            launch(kf, g2, kWG, 0, e.st, e.n, e.ldv, V(), nv, w(), e.coef1, e.part, e.nslot, g2,
                   e.ctrl, 2, e.cache_cols);
        }));
        if (e.timer) e.timer->end(2, j);
        k_finish<<<nv + 1, kWG, 0, e.st>>>(e.part, g2, nv, e.nslot, e.vscale, e.h2, e.coef2, 2,
                                           kHalf, e.nscale, e.sigma, e.ctrl, 2);
        launch(k_givens<true>, 1, kGT, 0, e.st, j, e.m, e.part, g2, e.nslot, e.h1, e.h2, e.H, e.cs,
               e.sn, e.g, e.vscale, e.sigma, e.hist, e.hist_cap, e.Hraw, e.cc, e.lag, e.ctrl, 2);
    }

    // Single-reduction CGS2 (FP64 bases only): step 0 is the two-sweep
    // variant's first projection; step j >= 1 is SpMV on q = w1_{j-1}, one
    // dot sweep, one reduction, the column/coefficient kernel and the update
    // sweep; after the last step one more dot sweep finalises column m-1.
    void step_dc(int j) const {
        if constexpr (std::is_same<VT, double>::value && std::is_same<WT, double>::value) {
            if (e.timer) e.timer->begin(0, j);
            if (j == 0) spmv_any<VT>(Vcol(0), e.vscale);
            else spmv_any<WT>(w(), nullptr);
            if (e.timer) e.timer->end(0, j);
            if (fused()) coarse_slots(e.s_step, 2);
            else coarse(y(), e.s_step, 2);
            if (j == 0) {
                if (e.timer) e.timer->begin(1, 0);
                auto kf = k_pass1<8, 1, VT, WT, AT, ACC>;
                const int g1 = grid_for((const void*)kf);
                launch(kf, g1, kWG, 0, e.st, e.n, e.ldv, V(), 1, y(), e.azrp, e.azci, azv(), e.azc1,
                       azv1(), e.s_step, e.R, w(), e.part, e.nslot, g1, e.ctrl, 2, e.cache_cols);
                if (e.timer) e.timer->end(1, 0);
                k_finish<<<2, kWG, 0, e.st>>>(e.part, g1, 1, e.nslot, e.vscale, e.h1, e.coef1, 1, kHalf,
                                              e.nscale, e.sigma, e.ctrl, 2);
                if (e.timer) e.timer->begin(2, 0);
                auto kf2 = k_pass2<8, 1, VT, WT, ACC>;
                const int g2 = grid_for((const void*)kf2);
                launch(kf2, g2, kWG, 0, e.st, e.n, e.ldv, V(), 1, w(), e.coef1, e.part, e.nslot, g2,
                       e.ctrl, 2, e.cache_cols);
                if (e.timer) e.timer->end(2, 0);
                k_finish<<<1, kWG, 0, e.st>>>(e.part, g2, 0, e.nslot, e.vscale, e.h2, e.coef2, 2, kHalf,
                                              e.nscale, e.sigma, e.ctrl, 2);
                return;
            }
            dc_dots<true>(j);
            GM_JMAX_SWITCH(j, VT, ({
                auto kf = k_dc_update<J, LanesForLag<J, VT>::value>;
                const int g = grid_for((const void*)kf);
                if (e.timer) e.timer->begin(2, j);
                launch(kf, g, kWG, 0, e.st, e.n, e.ldv, V(), j, w(), y(), e.coef1, e.coef2, e.lag,
                       e.ctrl, 2, e.cache_cols);
                if (e.timer) e.timer->end(2, j);
            }));
        }
    }

    // Dot sweep with nv = j, its reduction and the column kernel (U: with the
    // SpMV output; else the cycle's last column).
    template <bool UU>
    void dc_dots(int j) const {
        int g = 0;
        GM_JMAX_SWITCH(j, VT, ({
            auto kf = k_dc_dots<J, LanesForLag<J, VT>::value, UU>;
            g = grid_for((const void*)kf);
            if (e.timer) e.timer->begin(1, j);
            launch(kf, g, kWG, 0, e.st, e.n, e.ldv, (const double*)V(), j, (const double*)w(), (double*)y(),
                   e.azrp, e.azci, (const double*)azv(), e.azc1, (const double*)azv1(), e.s_step, e.R,
                   e.part, g, e.ctrl, 2, e.cache_cols);
            if (e.timer) e.timer->end(1, j);
        }));
        k_dc_sum<<<2 * j + 3, kWG, 0, e.st>>>(e.part, g, e.dcs, e.ctrl, 2);
        launch(k_dc_step<!UU>, 1, kGT, 0, e.st, j, e.m, (const double*)e.dcs, e.h1, e.H, e.cs, e.sn, e.g,
               e.vscale, (const double*)e.sigma, e.hist, e.hist_cap, e.Hraw, e.coef1, e.coef2, e.lag,
               e.ctrl, 2);
    }

    // y = scale * A x for the step's input vector x (type XT), with the fused
    // Z^T y partials when available.
    template <typename XT>
    void spmv_any(const XT* x, const double* scale) const {
        if (e.L == kSell)
            sell_launch<0, AT, XT, double, WT, ACC>(e, x, scale, nullptr, y(), 0, 2);
        else if (fused())
            stream_fused<0, AT, XT, double, WT, ACC>(e, vals(), x, scale, nullptr, y(), 0, 2);
        else
            spmv_dispatch<AT, XT, WT, ACC>(e.L, e.NB, e.st, e.n, e.rowptr, e.colind, vals(), x, scale,
                                           y(), e.ctrl, 2);
    }

    template <typename BT>
    void cycle(const BT* b) const {
        for (int j = 0; j < e.m; ++j) {
            if (e.dcgs) step_dc(j);
            else if (e.lagged) step_lag(j);
            else step(j);
        }
        if constexpr (std::is_same<VT, double>::value && std::is_same<WT, double>::value)
            if (e.dcgs) dc_dots<false>(e.m);
        k_backsolve<<<1, kWG, 0, e.st>>>(e.m, e.H, e.g, e.vscale, e.coef1, e.cyc_k, e.cyc_cap,
                                         e.ctrl, 1);
        bool adapted = false;
        if constexpr (std::is_same<VT, double>::value) {
            if (e.adapt) {
                adapt_cycle_end(e, V(), e.coef1);   // x += M^{-1} V_k y_k; new U, T
                adapted = true;
            }
        }
        if (!adapted) k_xupdate<VT><<<e.NB, kWG, 0, e.st>>>(e.n, e.ldv, V(), e.coef1, e.xh, e.ctrl, 1);
        restart_block(b, false, 0.0, 0.0);
    }
};

// Instantiated entry points (declared in internal.hpp).
void launch_restart_init(const EngineArgs& a, const void* b, double rtol, double r0_override) {
    switch (a.prec) {
        case kPrecF64: Engine<double, double, double, double>(a).restart_block((const double*)b, true, rtol, r0_override); break;
        case kPrecF32: Engine<float, float, float, float>(a).restart_block((const float*)b, true, rtol, r0_override); break;
        default: Engine<float, __half, float, float>(a).restart_block((const float*)b, true, rtol, r0_override); break;
    }
}

void launch_cycle(const EngineArgs& a, const void* b) {
    switch (a.prec) {
        case kPrecF64: Engine<double, double, double, double>(a).cycle((const double*)b); break;
        case kPrecF32: Engine<float, float, float, float>(a).cycle((const float*)b); break;
        default: Engine<float, __half, float, float>(a).cycle((const float*)b); break;
    }
}

template <typename AT, typename VT, typename WT, typename ACC>
static void pass_probe(const EngineArgs& e, int kind, int nv) {
    const VT* V = reinterpret_cast<const VT*>(e.V);
    WT* y = reinterpret_cast<WT*>(e.y);
    WT* w = reinterpret_cast<WT*>(e.w);
    if (kind == 1) {
        GM_JMAX_SWITCH(nv, VT, (k_pass1<J, T, VT, WT, AT, ACC><<<e.NB, kWG, 0, e.st>>>(
                                    e.n, e.ldv, V, nv, y, e.azrp, e.azci, (const AT*)e.azv, e.azc1,
                                    (const AT*)e.azv1, e.s_step, e.R, w, e.part, e.nslot, e.NB,
                                    nullptr, 0, e.cache_cols)));
    } else if (kind == 2) {
        GM_JMAX_SWITCH(nv, VT, (k_pass2<J, T, VT, WT, ACC><<<e.NB, kWG, 0, e.st>>>(
                                    e.n, e.ldv, V, nv, w, e.coef1, e.part, e.nslot, e.NB, nullptr, 0,
                                    e.cache_cols)));
    } else {
        GM_JMAX_SWITCH(nv, VT, (k_pass3<J, T, VT, WT, ACC><<<e.NB, kWG, 0, e.st>>>(
                                    e.n, e.ldv, (VT*)V, nv, w, e.coef2, e.sigma, e.part, e.nslot,
                                    e.NB, nullptr, 0, e.cache_cols)));
    }
}

// One launch of a pass kernel in the engine's precision (tuning probes).
void launch_pass_probe(const EngineArgs& e, int kind, int nv) {
    switch (e.prec) {
        case kPrecF64: pass_probe<double, double, double, double>(e, kind, nv); break;
        case kPrecF32: pass_probe<float, float, float, float>(e, kind, nv); break;
        default: pass_probe<float, __half, float, float>(e, kind, nv); break;
    }
}

void launch_correct(hipStream_t st, int NB, int n, const int* zrp, const int* zci, const double* zv,
                    const double* s, int R, const double* xh, double* x) {
    k_correct<<<NB, kWG, 0, st>>>(n, zrp, zci, zv, s, R, xh, x);
}

void launch_residual_f64(hipStream_t st, int L, int NB, int n, const int* rp, const int* ci,
                         const double* v, const double* x, const double* b, double* r, double* part,
                         int slot) {
    residual_dispatch<double, double, double, double>(L, NB, st, n, rp, ci, v, x, b, r, part, slot,
                                                      nullptr, 0);
}

void launch_sum_slot(hipStream_t st, const double* part, int NB, int slot, double* out) {
    k_sum_slot<<<1, kWG, 0, st>>>(part, NB, slot, out);
}

void launch_spmv_f64(hipStream_t st, int L, int NB, int n, const int* rp, const int* ci,
                     const double* v, const double* x, double* y) {
    spmv_dispatch<double, double, double, double>(L, NB, st, n, rp, ci, v, x, nullptr, y, nullptr, 0);
}

// Standalone FP64 sliced-ELL products (no fused Z^T y); wmax = widest row.
template <int MODE, int WMAX>
static void sell_f64(hipStream_t st, int NB, int n, const int* off, const int* perm, int wuni,
                     const short* col, const double* val, const double* x, const double* b, double* y,
                     double* part, int slot) {
    const int grid = MODE == 0 ? std::max(1, (n + kWG - 1) / kWG) : NB;
    k_spmv_sell<MODE, false, WMAX, kWG, double, double, double, double, double><<<grid, kWG, 0, st>>>(
        n, off, perm, wuni, col, val, x, nullptr, b, y, part, slot, NB, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
}

template <int MODE>
static void sell_f64_w(int wmax, hipStream_t st, int NB, int n, const int* off, const int* perm,
                       int wuni, const short* col, const double* val, const double* x,
                       const double* b, double* y, double* part, int slot) {
    if (wmax <= 9) sell_f64<MODE, 9>(st, NB, n, off, perm, wuni, col, val, x, b, y, part, slot);
    else if (wmax <= 12) sell_f64<MODE, 12>(st, NB, n, off, perm, wuni, col, val, x, b, y, part, slot);
    else if (wmax <= 16) sell_f64<MODE, 16>(st, NB, n, off, perm, wuni, col, val, x, b, y, part, slot);
    else if (wmax <= 25) sell_f64<MODE, 25>(st, NB, n, off, perm, wuni, col, val, x, b, y, part, slot);
    else sell_f64<MODE, 0>(st, NB, n, off, perm, wuni, col, val, x, b, y, part, slot);
}

void launch_spmv_sell_f64(hipStream_t st, int NB, int n, const int* off, const int* perm, int wuni,
                          int wmax, const short* col, const double* val, const double* x, double* y) {
    sell_f64_w<0>(wmax, st, NB, n, off, perm, wuni, col, val, x, nullptr, y, nullptr, 0);
}

void launch_residual_sell_f64(hipStream_t st, int NB, int n, const int* off, const int* perm,
                              int wuni, int wmax, const short* col, const double* val, const double* x,
                              const double* b, double* r, double* part, int slot) {
    sell_f64_w<1>(wmax, st, NB, n, off, perm, wuni, col, val, x, b, r, part, slot);
}

void launch_spmv_f32(hipStream_t st, int L, int NB, int n, const int* rp, const int* ci,
                     const float* v, const float* x, float* y) {
    spmv_dispatch<float, float, float, float>(L, NB, st, n, rp, ci, v, x, nullptr, y, nullptr, 0);
}

void launch_scale_to_f32(hipStream_t st, int NB, int n, const double* r, const double* nrm2,
                         float* out) {
    k_scale_to_f32<<<NB, kWG, 0, st>>>(n, r, nrm2, out);
}

void launch_axpy_norm(hipStream_t st, int NB, int n, const double* nrm2, const double* d, double* x) {
    k_axpy_norm<<<NB, kWG, 0, st>>>(n, nrm2, d, x);
}

void launch_ctrl_reset(hipStream_t st, Ctrl* c, int64_t max_iters, int64_t hist_base) {
    k_ctrl_reset<<<1, 64, 0, st>>>(c, max_iters, hist_base);
}

void launch_fill(hipStream_t st, double* p, int64_t n, double v) {
    const int64_t nb = std::min<int64_t>((n + kWG - 1) / kWG, 2048);
    if (nb > 0) k_fill<<<(int)nb, kWG, 0, st>>>(p, n, v);
}

void launch_copy(hipStream_t st, const double* a, double* b, int64_t n) {
    const int64_t nb = std::min<int64_t>((n + kWG - 1) / kWG, 2048);
    if (nb > 0) k_copy_f64<<<(int)nb, kWG, 0, st>>>(a, b, n);
}

GM_DEBUG_ACCESSOR(dbg_take_krylov)

}  // namespace gm
