// Block GMRES(m) for k <= 16 right-hand sides sharing A (A X = B).
//
// The paper solves one right-hand side at a time (Sec. 3.2); with several,
// the same minimisation over the block Krylov space span{R0, A R0, ...}
// turns the Gram-Schmidt work into tall-skinny matrix products, which run
// here on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
//   - vectors are 16-wide row-major panels (n_pad x 16, columns >= k zero):
//     one row of a panel is one 128-byte line;
//   - SpMM Y = A X: 16 lanes per row, one per column, so every gather reads
//     one line of X;
//   - C = [V_0 .. V_j]^T W: one 16x16 MFMA accumulator per panel, 4 rows of
//     every panel per instruction (one coalesced 512-byte load per panel);
//   - W -/+= sum_i V_i C_i: one 16-row tile per wavefront, the coefficients in
//     LDS;
//   - block Gram-Schmidt applied twice (BCGS2), then the new block by
//     Cholesky QR applied twice (CholQR2): H_{j+1,j} = R2 R1;
//   - the band Hessenberg least-squares problem by Householder reflections
//     updated per block step in one workgroup (the oracle refactors it from
//     scratch; equal in exact arithmetic), the per-column residual estimate
//     from the transformed right-hand side (analogue of eq. res).
// Readings shared with the oracle: iterations are block steps; a cycle runs on
// the columns whose true residual has not passed; a new column whose norm
// after orthogonalisation is <= 1e-10 times its norm before ends the cycle
// after that block step (its new basis block is never used); at a restart a
// residual column dependent on the earlier ones (same test) adds no basis
// vector but stays a right-hand side of the least-squares problem (kb <= ka
// basis columns per block); a zero initial residual column is rejected.
#include <hip/hip_ext.h>

#include <cmath>
#include <mutex>
#include <new>

#include "internal.hpp"

namespace gm {

namespace {

constexpr int kBW = 16;            // panel width
constexpr int kPan = kBW * kBW;    // entries of one 16 x 16 coefficient block
constexpr int kDotGrid = 1024;     // workgroups of the dot kernel (partials)
constexpr int kSplit = 16;         // first-level splits of the partial sums
constexpr int kNormGrid = 1024;    // workgroups of the residual kernel
constexpr int kLdH = (kBlockStepsMax + 1) * kBW;   // rows of the least-squares arrays
constexpr double kBdTol = 1e-10;
constexpr int kZtChunksMax = 64;   // workgroups per row of Z^T in the panel's Z^T W (at most)

typedef double d4 __attribute__((ext_vector_type(4)));

// D += A B for A 16x4, B 4x16: lane l feeds A[l % 16][l / 16] and
// B[l / 16][l % 16]; register r of lane l holds D[l / 16 + 4 r][l % 16].
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row-major n x k (caller layout) <-> panel of pw columns (pw = 8 or 16,
// k <= pw; rows of pw doubles).
__global__ __launch_bounds__(kWG) void k_bpack(int64_t n, int k, int pw, const double* __restrict__ src,
                                               double* __restrict__ P) {
    const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (e >= n * pw) return;
    const int64_t row = e / pw;
    const int c = (int)(e % pw);
    P[e] = (c < k && src) ? src[row * k + c] : 0.0;
}

__global__ __launch_bounds__(kWG) void k_bunpack(int64_t n, int k, int pw, const double* __restrict__ P,
                                                 double* __restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (e >= n * k) return;
    const int64_t row = e / k;
    const int c = (int)(e % k);
    dst[e] = P[row * pw + c];
}

// Deflation of a panel (Sec. 3.3, eq. precond1, applied to each of the 16
// columns): T = Z^T W, S = E^{-1} T, then W -= (A Z) S (projection) or
// X += Z S (coarse correction at exit, eq. precond2).
//
// Partial sums of T: workgroup (c, ch) sums chunk ch (of nch) of row c of
// Z^T, kWG / PW entries per round with one lane per panel column, four
// rounds' index loads issued before their gathers; fixed order.  Columns
// PW..15 of a partial are zero.
template <int PW>
__global__ __launch_bounds__(kWG) void k_bzt(int nch, const int* __restrict__ ztrp,
                                             const int* __restrict__ ztci, const double* __restrict__ ztv,
                                             const double* __restrict__ W, double* __restrict__ zpart,
                                             const int* __restrict__ stop) {
    constexpr int RG = kWG / PW;   // entries per round
    constexpr int U = 4;
    __shared__ double red[kWG];
    if (stop && *stop) return;   // a later step of a cycle that has ended
    const int c = blockIdx.x, ch = blockIdx.y;
    const int q0 = ztrp[c], q1 = ztrp[c + 1];
    const int cl = (q1 - q0 + nch - 1) / nch;
    const int a0 = q0 + ch * cl, a1 = min(q1, a0 + cl);
    const int l = threadIdx.x & (PW - 1), g = threadIdx.x / PW;
    double acc = 0.0;
    for (int q = a0 + g; q < a1; q += U * RG) {
        int row[U];
        double zvv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int qu = q + u * RG;
            row[u] = qu < a1 ? ztci[qu] : 0;
            zvv[u] = qu < a1 ? ztv[qu] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += zvv[u] * W[(int64_t)row[u] * PW + l];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < kBW) {
        double t = 0.0;
        if (threadIdx.x < PW)
            for (int i = 0; i < RG; ++i) t += red[i * PW + threadIdx.x];
        zpart[((int64_t)c * nch + ch) * kBW + threadIdx.x] = t;
    }
}

// S = E^{-1} T (R x 16, row c of T the sum of its chunks in order); one
// workgroup, T and E^{-1} staged in LDS.
__global__ __launch_bounds__(kWG) void k_bcoarse(int R, int nch, const double* __restrict__ zpart,
                                                 const double* __restrict__ Einv, double* __restrict__ S,
                                                 const int* __restrict__ stop) {
    __shared__ double T[kBlockZMax * kBW];
    __shared__ double Ei[kBlockZMax * kBlockZMax];
    if (stop && *stop) return;
    for (int e = threadIdx.x; e < R * kBW; e += kWG) {
        const int c = e / kBW, l = e % kBW;
        double t = 0.0;
        for (int ch = 0; ch < nch; ++ch) t += zpart[((int64_t)c * nch + ch) * kBW + l];
        T[e] = t;
    }
    for (int e = threadIdx.x; e < R * R; e += kWG) Ei[e] = Einv[e];
    __syncthreads();
    for (int e = threadIdx.x; e < R * kBW; e += kWG) {
        const int i = e / kBW, l = e % kBW;
        double t = 0.0;
        for (int a = 0; a < R; ++a) t += Ei[a * R + i] * T[a * kBW + l];
        S[e] = t;
    }
}

// P += sign * M S over the rows of the CSR matrix M (n x R, local columns):
// sign -1 with M = A Z projects W, sign +1 with M = Z corrects X.  PW lanes
// per row (one per panel column), S (R x 16) staged in LDS.
template <int PW>
__global__ __launch_bounds__(kWG) void k_bzapply(int64_t n, int R, const int* __restrict__ mrp,
                                                 const int* __restrict__ mci, const double* __restrict__ mv,
                                                 const double* __restrict__ S, double sign, double* __restrict__ P,
                                                 const int* __restrict__ stop) {
    constexpr int rpr = kWG / PW;   // rows per round
    __shared__ double Ss[kBlockZMax * kBW];
    if (stop && *stop) return;
    for (int e = threadIdx.x; e < R * kBW; e += kWG) Ss[e] = S[e];
    __syncthreads();
    const int l = threadIdx.x & (PW - 1), rl = threadIdx.x / PW;
    for (int64_t r0 = (int64_t)blockIdx.x * rpr; r0 < n; r0 += (int64_t)gridDim.x * rpr) {
        const int64_t row = r0 + rl;
        if (row >= n) continue;
        double t = 0.0;
        for (int q = mrp[row]; q < mrp[row + 1]; ++q) {
            GM_DCHECK(mci[q] >= 0 && mci[q] < R, kDbgBlockCol);
            t += mv[q] * Ss[mci[q] * kBW + l];
        }
        P[row * PW + l] += sign * t;
    }
}

// Per-workgroup partial sums of squares of the 16 columns of a panel.
__global__ __launch_bounds__(kWG) void k_bnorm(int64_t n, int pw, const double* __restrict__ W,
                                               double* __restrict__ part) {
    __shared__ double red[kWG];
    const int l = threadIdx.x & (kBW - 1), rl = threadIdx.x / kBW;
    double acc = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * (kWG / kBW); r0 < n; r0 += (int64_t)gridDim.x * (kWG / kBW)) {
        const int64_t row = r0 + rl;
        if (row < n && l < pw) {
            const double y = W[row * pw + l];
            acc += y * y;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < kBW) {
        double t = 0.0;
        for (int i = 0; i < kWG / kBW; ++i) t += red[i * kBW + threadIdx.x];
        part[(int64_t)blockIdx.x * kBW + threadIdx.x] = t;
    }
}

// Y = A X (MODE 0), or Y = B - A X with per-workgroup partial sums of squares
// of every column (MODE 1).  16 lanes per row, 16 rows per workgroup.
template <int MODE, int PW>
__global__ __launch_bounds__(kWG) void k_bspmm(int64_t n, const int* __restrict__ rowptr,
                                               const int* __restrict__ colind,
                                               const double* __restrict__ vals,
                                               const double* __restrict__ X,
                                               const double* __restrict__ B, double* __restrict__ Y,
                                               double* __restrict__ part, const int* __restrict__ stop) {
    __shared__ double red[kWG];
    if (stop && *stop) return;   // a later step of a cycle that has ended
    // PW lanes per row (one per panel column), kWG / PW rows per round.
    constexpr int pw = PW, rpr = kWG / PW;
    const int c = threadIdx.x & (pw - 1), rl = threadIdx.x / pw;
    double nrm = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * rpr; r0 < n; r0 += (int64_t)gridDim.x * rpr) {
        const int64_t row = r0 + rl;
        if (row < n) {
            const int q0 = rowptr[row], q1 = rowptr[row + 1];
            double acc = 0.0;
            int q = q0;
            for (; q + 4 <= q1; q += 4) {
                const int c0 = colind[q], c1 = colind[q + 1], c2 = colind[q + 2], c3 = colind[q + 3];
                GM_DCHECK(min(min(c0, c1), min(c2, c3)) >= 0 && max(max(c0, c1), max(c2, c3)) < n,
                          kDbgBlockCol);
                const double a0 = vals[q], a1 = vals[q + 1], a2 = vals[q + 2], a3 = vals[q + 3];
                const double x0 = X[(int64_t)c0 * pw + c], x1 = X[(int64_t)c1 * pw + c];
                const double x2 = X[(int64_t)c2 * pw + c], x3 = X[(int64_t)c3 * pw + c];
                acc += a0 * x0;
                acc += a1 * x1;
                acc += a2 * x2;
                acc += a3 * x3;
            }
            for (; q < q1; ++q) {
                GM_DCHECK(colind[q] >= 0 && colind[q] < n, kDbgBlockCol);
                acc += vals[q] * X[(int64_t)colind[q] * pw + c];
            }
            if (MODE == 0) {
                Y[row * pw + c] = acc;
            } else {
                const double y = B[row * pw + c] - acc;
                Y[row * pw + c] = y;
                nrm += y * y;
            }
        }
    }
    if (MODE == 1) {
        red[threadIdx.x] = nrm;
        __syncthreads();
        if (threadIdx.x < kBW) {
            double s = 0.0;
            if (threadIdx.x < pw)
                for (int i = 0; i < rpr; ++i) s += red[i * pw + threadIdx.x];
            part[(int64_t)blockIdx.x * kBW + threadIdx.x] = s;
        }
    }
}

// Column sums of squares: out[c] = sum_b part[b * 16 + c].
__global__ __launch_bounds__(kWG) void k_bcolsum(int nblk, const double* __restrict__ part,
                                                 double* __restrict__ out) {
    __shared__ double red[kWG];
    const int c = threadIdx.x & (kBW - 1), s = threadIdx.x / kBW;
    double acc = 0.0;
    for (int b = s; b < nblk; b += kWG / kBW) acc += part[(int64_t)b * kBW + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < kBW) {
        double t = 0.0;
        for (int i = 0; i < kWG / kBW; ++i) t += red[i * kBW + threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// Partial products C_i = P_i^T W (P_i = panel i of V for i < nv; with gram,
// P_nv = W) over 4-row chunks, one MFMA accumulator per panel; workgroups
// with blockIdx.y = g take panels [NG g, NG g + NG) (W is read once per
// group, which keeps NG accumulators per lane and the occupancy high);
// per-workgroup partials part[(blockIdx.x * nb + i) * 256 + m * 16 + n]
// (fixed order).  Panels beyond nb are loaded (W again) and multiplied but
// never stored, so the loop body is branch-free.
// Entry t of a workgroup's 16 x 16 block of partial dots from the
// wavefronts' accumulators red[w] (row-major).  16-wide panels: the sum over
// the wavefronts.  8-wide panels (lanes l%16 >= 8 on the second half of each
// 8-row run): entry (i, j) < 8 is quadrant (i, j) plus quadrant (i+8, j+8);
// the other entries are zero, as the 16-wide layout leaves them.
template <int PW>
__device__ __forceinline__ double fold_partial(const double (*red)[kPan], int t) {
    double s = 0.0;
    if (PW == 16) {
#pragma unroll
        for (int w = 0; w < kWG / kWave; ++w) s += red[w][t];
    } else if (t / kBW < 8 && t % kBW < 8) {
#pragma unroll
        for (int w = 0; w < kWG / kWave; ++w) s += red[w][t] + red[w][t + 8 * kBW + 8];
    }
    return s;
}

template <int NG, int PW>
__global__ __launch_bounds__(kWG) void k_bdots(int64_t n_pad, int64_t ps, const double* __restrict__ V,
                                               int nv, const double* __restrict__ W, int gram,
                                               double* __restrict__ part, const int* __restrict__ stop) {
    __shared__ double red[kWG / kWave][kPan];
    if (stop && *stop) return;   // a later step of a cycle that has ended

    const int l = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int nb = nv + gram, i0 = blockIdx.y * NG;
    d4 acc[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    const double* src[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) src[i] = i0 + i < nv ? V + (i0 + i) * ps : W;
    // 16-wide panels: lane l holds row r0 + l/16, column l%16, four rows a
    // step.  8-wide panels: lanes with l%16 >= 8 take the next four rows,
    // row r0 + l/16 + 4, column l%16 - 8, so a step covers eight whole rows
    // (one contiguous 512-byte run) with no idle lane; the 8x8 diagonal
    // quadrants of the accumulator then hold the products of the two row
    // halves (the off-diagonal quadrants mix them and are dropped), and their
    // sum is the 8x8 block of dots.
    constexpr int pw = PW;
    constexpr int rows = PW == 8 ? 8 : 4;   // rows per step and wavefront
    const int64_t e = PW == 8 ? (int64_t)(l / kBW + 4 * ((l & (kBW - 1)) >> 3)) * pw + (l & 7)
                              : (int64_t)(l / kBW) * pw + (l & (kBW - 1));
    const int64_t nw = (int64_t)gridDim.x * (kWG / kWave);
    for (int64_t r0 = ((int64_t)blockIdx.x * (kWG / kWave) + wv) * rows; r0 < n_pad; r0 += nw * rows) {
        const double b = W[r0 * pw + e];
        double a[NG];
#pragma unroll
        for (int i = 0; i < NG; ++i) a[i] = src[i][r0 * pw + e];
#pragma unroll
        for (int i = 0; i < NG; ++i) acc[i] = mfma16(a[i], b, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        if (i0 + i < nb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wv][(l / kBW + 4 * r) * kBW + (l & (kBW - 1))] = acc[i][r];
            __syncthreads();
            part[((int64_t)blockIdx.x * nb + i0 + i) * kPan + threadIdx.x] = fold_partial<PW>(red, threadIdx.x);
            __syncthreads();
        }
    }
}

// Sum of the dot partials over the workgroups, fixed order: a workgroup
// takes 16 entries; its 16 x 16 threads each sum split s (workgroups s,
// s + 16, ...) of one entry, then the splits are added in order.  out = the
// sums; with acc_into: acc_into[e] = (first ? 0 : acc_into[e]) + out[e] for
// e < acc_cnt, and (diag_blk >= 0) the diagonal of block diag_blk saved to
// nb2.
__global__ __launch_bounds__(kWG) void k_breduce(int nblk, int cnt, const double* __restrict__ part,
                                                 double* __restrict__ out, double* acc_into, int acc_cnt,
                                                 int first, int diag_blk, double* __restrict__ nb2,
                                                 const int* __restrict__ stop) {
    static_assert(kSplit * kBW == kWG, "16 entries x 16 splits per workgroup");
    __shared__ double ps[kSplit][kBW + 1];
    if (stop && *stop) return;   // a later step of a cycle that has ended
    const int el = threadIdx.x % kBW, sp = threadIdx.x / kBW;
    const int e = blockIdx.x * kBW + el;
    double acc = 0.0;
    if (e < cnt) {
#pragma unroll 8
        for (int b = sp; b < nblk; b += kSplit) acc += part[(int64_t)b * cnt + e];
    }
    ps[sp][el] = acc;
    __syncthreads();
    if (sp == 0 && e < cnt) {
        double a = 0.0;
        for (int q = 0; q < kSplit; ++q) a += ps[q][el];
        out[e] = a;
        if (acc_into && e < acc_cnt) acc_into[e] = (first ? 0.0 : acc_into[e]) + a;
        if (nb2 && diag_blk >= 0) {
            const int d = e - diag_blk * kPan;
            if (d >= 0 && d < kPan && d / kBW == d % kBW) nb2[d / kBW] = a;
        }
    }
}

// sum_{i < nb} P_i C_i over the 16-row tile at r0 (C_i row-major 16 x 16 in
// LDS): lane l feeds row r0 + l%16, columns l/16 + 4q of each panel (the
// MFMA A operand, pw/4 steps a panel) and comes out holding rows
// r0 + l/16 + 4r, column l%16.  For 8-wide panels the B operand repeats C's
// first 8 columns in its upper 8, so both halves of the result hold the tile.
template <int PW>
__device__ __forceinline__ d4 tile_product(const double* V, int64_t ps, int nb, const double* cs, int64_t r0,
                                           int l) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const int col = PW == 8 ? (l & 7) : (l & (kBW - 1));
    for (int i = 0; i < nb; ++i) {
        const double* P = V + i * ps + (r0 + (l & (kBW - 1))) * PW + l / kBW;
        const double* Ci = cs + i * kPan + (l / kBW) * kBW + col;
        double a[PW / 4], b[PW / 4];
#pragma unroll
        for (int q = 0; q < PW / 4; ++q) {
            a[q] = P[4 * q];
            b[q] = Ci[4 * q * kBW];
        }
#pragma unroll
        for (int q = 0; q < PW / 4; ++q) acc = mfma16(a[q], b[q], acc);
    }
    return acc;
}

// OUT = IN + sign * sum_{i < nb} P_i C_i (P_i = panel i of V, C_i = C[i*256 ..]
// row-major 16x16, staged in nb * 2 KB of dynamic LDS given at launch), one
// 16-row tile per wavefront; IN may be NULL; IN, OUT and the panels may alias
// (a tile is read completely before it is written, by the same wavefront).
template <int PW>
__global__ __launch_bounds__(kWG) void k_bgemm(int64_t n_pad, int64_t ps, const double* V, int nb,
                                               const double* __restrict__ C, const double* IN,
                                               double sign, double* OUT, const int* __restrict__ stop) {
    if (stop && *stop) return;   // a later step of a cycle that has ended
    constexpr int pw = PW;
    extern __shared__ double cs[];   // nb coefficient blocks (dynamic)
    for (int t = threadIdx.x; t < nb * kPan; t += kWG) cs[t] = C[t];
    __syncthreads();
    const int l = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t ntile = n_pad / kBW;
    for (int64_t tile = (int64_t)blockIdx.x * (kWG / kWave) + wv; tile < ntile;
         tile += (int64_t)gridDim.x * (kWG / kWave)) {
        const int64_t r0 = tile * kBW;
        d4 acc = tile_product<PW>(V, ps, nb, cs, r0, l);
        if (PW == 8) {
            // both column halves of the accumulator hold the tile; lane l
            // stores rows r0 + l/16 + 4 h + 8 s (h = its half, s = 0, 1)
            const int h = (l & (kBW - 1)) >> 3;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int64_t idx = (r0 + l / kBW + 4 * (2 * s + h)) * pw + (l & 7);
                OUT[idx] = (IN ? IN[idx] : 0.0) + sign * (h ? acc[2 * s + 1] : acc[2 * s]);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t idx = (r0 + l / kBW + 4 * r) * pw + (l & (kBW - 1));
                OUT[idx] = (IN ? IN[idx] : 0.0) + sign * acc[r];
            }
        }
    }
}

// First projection and second dot pass of BCGS2 in one sweep over the basis:
// OUT = IN - sum_{i < nb} P_i C_i (as k_bgemm with sign -1), then the partial
// dots P_i^T OUT of this workgroup's tiles (as k_bdots, no Gram block).  One
// 16-row tile per wavefront; the product reads each panel's tile with lane l
// holding row r0 + l%16, columns l/16 + 4q (MFMA A operand), and the new tile
// comes out with lane l holding rows r0 + l/16 + 4r, column l%16 -- the B
// operand layout of the dot products -- so only the panels' tiles are read a
// second time for the dots, in that layout, right after the first read
// (from the caches).  nb <= NBMAX accumulators per lane.  The 16-wide
// instance is held to 128 registers (four wavefronts per SIMD, no spills);
// the 8-wide one would spill there and keeps three.
template <int NBMAX, int PW>
__global__ __launch_bounds__(kWG, PW == 16 ? 4 : 1) void k_bgemm_dots(int64_t n_pad, int64_t ps, const double* V,
                                                                     int nb,
                                                    const double* __restrict__ C, const double* IN,
                                                    double* OUT, double* __restrict__ part,
                                                    const int* __restrict__ stop) {
    if (stop && *stop) return;   // a later step of a cycle that has ended
    constexpr int pw = PW;
    __shared__ double cs[NBMAX * kPan];
    __shared__ double red[kWG / kWave][kPan];
    for (int t = threadIdx.x; t < nb * kPan; t += kWG) cs[t] = C[t];
    __syncthreads();
    const int l = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    d4 dacc[NBMAX];
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) dacc[i] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t ntile = n_pad / kBW;
    for (int64_t tile = (int64_t)blockIdx.x * (kWG / kWave) + wv; tile < ntile;
         tile += (int64_t)gridDim.x * (kWG / kWave)) {
        const int64_t r0 = tile * kBW;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        const int col = PW == 8 ? (l & 7) : (l & (kBW - 1));   // 8-wide: C's columns repeated
#pragma unroll
        for (int i = 0; i < NBMAX; ++i) {
            if (i < nb) {
                const double* P = V + i * ps + (r0 + (l & (kBW - 1))) * pw + l / kBW;
                const double* Ci = cs + i * kPan + (l / kBW) * kBW + col;
                double a[PW / 4], b[PW / 4];
#pragma unroll
                for (int q = 0; q < PW / 4; ++q) {
                    a[q] = P[4 * q];
                    b[q] = Ci[4 * q * kBW];
                }
#pragma unroll
                for (int q = 0; q < PW / 4; ++q) acc = mfma16(a[q], b[q], acc);
            }
        }
        if (PW == 8) {
            // Both halves of acc hold the tile.  Lane l takes rows
            // r0 + l/16 + 4 h + 8 s (h = its column half, s = 0, 1), column
            // l%8: two contiguous 8-row runs, and for each s the dot step's
            // operands in the layout k_bdots uses for 8-wide panels.
            const int h = (l & (kBW - 1)) >> 3;
            double wn[2];
            int64_t idx[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                idx[s] = (r0 + l / kBW + 4 * (2 * s + h)) * pw + (l & 7);
                wn[s] = IN[idx[s]] - (h ? acc[2 * s + 1] : acc[2 * s]);
                OUT[idx[s]] = wn[s];
            }
#pragma unroll
            for (int i = 0; i < NBMAX; ++i) {
                if (i < nb) {
                    const double* P = V + i * ps;
                    const double a0 = P[idx[0]], a1 = P[idx[1]];
                    dacc[i] = mfma16(a0, wn[0], dacc[i]);
                    dacc[i] = mfma16(a1, wn[1], dacc[i]);
                }
            }
        } else {
            double wn[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t idx = (r0 + l / kBW + 4 * r) * pw + (l & (kBW - 1));
                wn[r] = IN[idx] - acc[r];
                OUT[idx] = wn[r];
            }
#pragma unroll
            for (int i = 0; i < NBMAX; ++i) {
                if (i < nb) {
                    const double* P = V + i * ps + (r0 + l / kBW) * pw + (l & (kBW - 1));
                    double a[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) a[r] = P[4 * r * pw];
#pragma unroll
                    for (int r = 0; r < 4; ++r) dacc[i] = mfma16(a[r], wn[r], dacc[i]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
        if (i < nb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wv][(l / kBW + 4 * r) * kBW + (l & (kBW - 1))] = dacc[i][r];
            __syncthreads();
            part[((int64_t)blockIdx.x * nb + i) * kPan + threadIdx.x] = fold_partial<PW>(red, threadIdx.x);
            __syncthreads();
        }
    }
}

// OUT = IN + sign * sum_{i < nb} P_i C_i (as k_bgemm), then the partial Gram
// block OUT^T OUT of this workgroup's tiles.  The new tile leaves the product
// in the layout both operands of the dot step take (as in k_bgemm_dots), so
// the Gram block needs no second read of OUT.  One 16-row tile per wavefront;
// the coefficients' LDS (sized for max(nb, kWG / kWave) blocks at launch)
// holds the wavefronts' accumulators at the end.
template <int PW>
__global__ __launch_bounds__(kWG) void k_bgemm_gram(int64_t n_pad, int64_t ps, const double* V, int nb,
                                                    const double* __restrict__ C, const double* IN, double sign,
                                                    double* OUT, double* __restrict__ part,
                                                    const int* __restrict__ stop) {
    if (stop && *stop) return;   // a later step of a cycle that has ended
    constexpr int pw = PW;
    extern __shared__ double cs[];   // max(nb, 4) blocks (dynamic): coefficients, then accumulators
    for (int t = threadIdx.x; t < nb * kPan; t += kWG) cs[t] = C[t];
    __syncthreads();
    const int l = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    d4 g = {0.0, 0.0, 0.0, 0.0};
    const int64_t ntile = n_pad / kBW;
    for (int64_t tile = (int64_t)blockIdx.x * (kWG / kWave) + wv; tile < ntile;
         tile += (int64_t)gridDim.x * (kWG / kWave)) {
        const int64_t r0 = tile * kBW;
        const d4 acc = tile_product<PW>(V, ps, nb, cs, r0, l);
        if (PW == 8) {
            // lane l: rows r0 + l/16 + 4 h + 8 s, column l%8 (h = its column
            // half); each s is one 8-row Gram step in the k_bdots layout
            const int h = (l & (kBW - 1)) >> 3;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int64_t idx = (r0 + l / kBW + 4 * (2 * s + h)) * pw + (l & 7);
                const double v = (IN ? IN[idx] : 0.0) + sign * (h ? acc[2 * s + 1] : acc[2 * s]);
                OUT[idx] = v;
                g = mfma16(v, v, g);
            }
        } else {
            double v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t idx = (r0 + l / kBW + 4 * r) * pw + (l & (kBW - 1));
                v[r] = (IN ? IN[idx] : 0.0) + sign * acc[r];
                OUT[idx] = v[r];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) g = mfma16(v[r], v[r], g);
        }
    }
    __syncthreads();   // every wavefront is done with the coefficients
    double (*red)[kPan] = reinterpret_cast<double (*)[kPan]>(cs);
#pragma unroll
    for (int r = 0; r < 4; ++r) red[wv][(l / kBW + 4 * r) * kBW + (l & (kBW - 1))] = g[r];
    __syncthreads();
    part[(int64_t)blockIdx.x * kPan + threadIdx.x] = fold_partial<PW>(red, threadIdx.x);
}

// R^T R = G for the 16x16 Gram matrix G (row-major); rows/columns >= k are
// the identity.  Rinv = R^{-1}; Rout = R Rprev (Rprev NULL: R).  With test,
// a pivot <= kBdTol times the column's norm before orthogonalisation
// (sqrt(nb2[c]), else sqrt(G_cc)) sets *flag |= 2, bdmask[c] = 1, and makes
// row c of R and of R^{-1} zero (the column counts as dependent).
__global__ void k_bchol(int k, const double* __restrict__ G, const double* __restrict__ nb2, int test,
                        const double* __restrict__ Rprev, double* __restrict__ Rout,
                        double* __restrict__ Rinv, int* flag, int* __restrict__ bdmask,
                        const int* __restrict__ stop) {
    if (stop && *stop) return;   // a later step of a cycle that has ended
    __shared__ double R[kPan], Ri[kPan], Gs[kPan], Rp[kPan], nbs[kBW];
    __shared__ int bd[kBW];
    const int t = threadIdx.x;   // 64 threads; t < 16 active in the triangular loops
    // Every input is read into LDS once, before the dependent loops.
    if (t < kBW) {
        bd[t] = 0;
        nbs[t] = nb2 ? nb2[t] : 0.0;
    }
    for (int e = t; e < kPan; e += blockDim.x) {
        R[e] = 0.0;
        Ri[e] = 0.0;
        Gs[e] = G[e];
        Rp[e] = Rprev ? Rprev[e] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < kBW; ++j) {
        if (t == 0) {
            double d;
            if (j >= k) {
                d = 1.0;
            } else {
                double p = Gs[j * kBW + j];
                for (int i = 0; i < j; ++i) p -= R[i * kBW + j] * R[i * kBW + j];
                const double before = nb2 ? nbs[j] : Gs[j * kBW + j];
                if (test && !(p > kBdTol * kBdTol * before)) bd[j] = 1;
                // A broken column counts as dependent: zero row of R.
                d = (p > 0.0 && !bd[j]) ? sqrt(p) : 0.0;
            }
            R[j * kBW + j] = d;
        }
        __syncthreads();
        if (t > j && t < kBW) {
            double s = (j < k && t < k) ? Gs[j * kBW + t] : 0.0;
            for (int i = 0; i < j; ++i) s -= R[i * kBW + j] * R[i * kBW + t];
            const double d = R[j * kBW + j];
            R[j * kBW + t] = d > 0.0 ? s / d : 0.0;
        }
        __syncthreads();
    }
    // Column t of R^{-1} by back substitution (broken pivots give zeros).
    if (t < kBW) {
        for (int i = kBW - 1; i >= 0; --i) {
            double s = i == t ? 1.0 : 0.0;
            for (int q = i + 1; q < kBW; ++q) s -= R[i * kBW + q] * Ri[q * kBW + t];
            const double d = R[i * kBW + i];
            Ri[i * kBW + t] = (d > 0.0 && !bd[i]) ? s / d : 0.0;
        }
    }
    __syncthreads();
    if (t < kBW) {
        for (int i = 0; i < kBW; ++i) {
            double o;
            if (Rprev) {
                o = 0.0;
                for (int q = i; q <= t; ++q) o += R[i * kBW + q] * Rp[q * kBW + t];
            } else {
                o = R[i * kBW + t];
            }
            Rout[i * kBW + t] = o;
            Rinv[i * kBW + t] = Ri[i * kBW + t];
        }
    }
    __syncthreads();
    if (t < kBW && test && bdmask) bdmask[t] = bd[t];
    if (t == 0 && test) {
        int any = 0;
        for (int j = 0; j < kBW; ++j) any |= bd[j];
        if (any) *flag |= 2;
    }
}

// In-place column selection of a panel: column i <- column map[i] (map[i] < 0:
// zero), one entry per thread.  pw divides the wavefront, so a row lies in
// one wavefront, whose loads of the row complete before any of its stores.
__global__ __launch_bounds__(kWG) void k_bselect(int64_t n, int pw, const int* __restrict__ map, double* P) {
    const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (e >= n * pw) return;
    const int c = (int)(e % pw);
    const int q = map[c];
    const double v = q >= 0 && q < pw ? P[e - c + q] : 0.0;
    P[e] = v;
}

// X[:, act[c]] += T[:, c] for c < ka.
__global__ __launch_bounds__(kWG) void k_bscatter(int64_t n, int pw, int ka, const int* __restrict__ act,
                                                  const double* __restrict__ T, double* __restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (e >= n * pw) return;
    const int64_t row = e / pw;
    const int c = (int)(e % pw);
    if (c < ka) X[row * pw + act[c]] += T[e];
}

// Least-squares state, column-major with kLdH rows: H (transformed Hbar),
// reflectors v (k + 1 entries per column) and beta, G (transformed [S; 0]).
struct LsView {
    double* H;      // kLdH * (kBlockStepsMax * kBW)
    double* v;      // (kBlockStepsMax * kBW) * (kBW + 1)
    double* beta;   // kBlockStepsMax * kBW
    double* G;      // kLdH * kBW
    double* rho0;   // kBW
    double* est;    // kBW
};

// G = [S; 0] for the cycle's starting block (S kb x ka, row-major in 16x16).
__global__ __launch_bounds__(kWG) void k_bls_init(int kb, int ka, const double* __restrict__ S, LsView ls) {
    for (int e = threadIdx.x; e < kLdH * kBW; e += kWG) {
        const int c = e / kLdH, i = e % kLdH;
        ls.G[e] = (c < ka && i < kb) ? S[i * kBW + c] : 0.0;
    }
}

// Block step j (k basis columns per block, ka right-hand sides): append the
// block column (rows 0 .. (j+2)k-1) built from the accumulated projection
// coefficients Csum (blocks 0..j) and H_{j+1,j} = Rj, apply the previous
// reflectors, make k new ones, apply them to G, and estimate each right-hand
// side's residual.  flag[0] |= 1 when every one passes.  It ends the block
// step: flag[2] counts the cycle's steps, and flag[1] (the gate of every later
// kernel of the cycle) is set once flag[0] is (this step ended the cycle).
__global__ __launch_bounds__(kWG) void k_bls(int j, int k, int ka, double rtol,
                                             const double* __restrict__ Csum,
                                             const double* __restrict__ Rj, LsView ls, int* flag) {
    if (flag[1]) return;   // a later step of a cycle that has ended
    // Columns padded by one entry: threads that walk different columns at
    // the same row then hit different LDS banks.
    __shared__ double h[kBW][kLdH + 1];
    __shared__ double vl[(kBlockStepsMax - 1) * kBW * (kBW + 1)];   // previous reflectors
    __shared__ double bl[(kBlockStepsMax - 1) * kBW];
    __shared__ double vs[kBW + 1];
    __shared__ double bs;
    // Rows c0 .. c0 + 2k - 1 of the right-hand sides' columns of G: the only
    // rows this step's reflectors touch, kept in LDS until the end.
    __shared__ double gl[kBW][2 * kBW + 1];
    __shared__ double est2[kBW];
    const int t = threadIdx.x;
    const int rows = (j + 2) * k, c0 = j * k;
    for (int e = t; e < kBW * 2 * kBW; e += kWG) {
        const int c = e / (2 * kBW), r = e % (2 * kBW);
        gl[c][r] = (c < ka && r < 2 * k) ? ls.G[(int64_t)c * kLdH + c0 + r] : 0.0;
    }
    // Every global load of the inputs is issued before the first is stored
    // to LDS (fixed trip counts, registers in between).
    constexpr int kVIt = ((kBlockStepsMax - 1) * kBW * (kBW + 1) + kWG - 1) / kWG;
    constexpr int kHIt = (kBW * kLdH + kWG - 1) / kWG;
    double vr[kVIt], hr[kHIt];
#pragma unroll
    for (int u = 0; u < kVIt; ++u) {
        const int e = t + u * kWG;
        vr[u] = e < c0 * (kBW + 1) ? ls.v[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kHIt; ++u) {
        const int e = t + u * kWG;
        const int col = e / kLdH, row = e % kLdH;
        double val = 0.0;
        if (e < kBW * kLdH && col < k && row < rows) {
            const int blk = row / k, kk = row % k;
            if (blk <= j) val = Csum[blk * kPan + kk * kBW + col];
            else val = kk <= col ? Rj[kk * kBW + col] : 0.0;
        }
        hr[u] = val;
    }
    for (int e = t; e < c0; e += kWG) bl[e] = ls.beta[e];
#pragma unroll
    for (int u = 0; u < kVIt; ++u) {
        const int e = t + u * kWG;
        if (e < c0 * (kBW + 1)) vl[e] = vr[u];
    }
#pragma unroll
    for (int u = 0; u < kHIt; ++u) {
        const int e = t + u * kWG;
        if (e < kBW * kLdH) h[e / kLdH][e % kLdH] = hr[u];
    }
    __syncthreads();
    // Previous reflectors, in order, on every column of the new block: 16
    // lanes per column, lane i holding entry p + i of reflector p's window
    // (lane 0 also entry p + 16 when k = 16); the dot product by shuffles
    // inside the 16-lane group.  Each group walks its own column, so the
    // groups need no barrier between reflectors.
    {
        const int ct = t / kBW, li = t & (kBW - 1);
        if (ct < k) {
            for (int p = 0; p < c0; ++p) {
                const double* vp = vl + p * (kBW + 1);
                const double v0 = li <= k ? vp[li] : 0.0;
                const double v16 = (li == 0 && k == kBW) ? vp[kBW] : 0.0;
                const double h0 = h[ct][p + li];
                const double h16 = (li == 0 && k == kBW) ? h[ct][p + kBW] : 0.0;
                double part = v0 * h0 + v16 * h16;
#pragma unroll
                for (int o = kBW / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, kBW);
                const double sp = part * bl[p];
                if (li <= k) h[ct][p + li] = h0 - sp * v0;
                if (li == 0 && k == kBW) h[ct][p + kBW] = h16 - sp * v16;
            }
        }
    }
    __syncthreads();
    // New reflectors, one per column of the block, each built by the first
    // 16 lanes (entries as above, norms by shuffles) and applied to the
    // block's later columns and to the right-hand sides by 16-lane groups.
    const int ct = t / kBW, li = t & (kBW - 1);
    for (int q = 0; q < k; ++q) {
        const int col = c0 + q;
        if (t < kBW) {
            const double x0 = li <= k ? h[q][col + li] : 0.0;
            const double x16 = (li == 0 && k == kBW) ? h[q][col + kBW] : 0.0;
            double n2 = x0 * x0 + x16 * x16;
#pragma unroll
            for (int o = kBW / 2; o > 0; o >>= 1) n2 += __shfl_xor(n2, o, kBW);
            const double nrm = sqrt(n2);
            const double a0 = __shfl(x0, 0, kBW);
            const double alpha = a0 >= 0.0 ? -nrm : nrm;
            const double w0 = nrm > 0.0 ? (li == 0 ? a0 - alpha : x0) : 0.0;
            const double w16 = nrm > 0.0 ? x16 : 0.0;
            double vv = w0 * w0 + w16 * w16;
#pragma unroll
            for (int o = kBW / 2; o > 0; o >>= 1) vv += __shfl_xor(vv, o, kBW);
            const double beta = (nrm > 0.0 && vv > 0.0) ? 2.0 / vv : 0.0;
            if (li <= k) {
                vs[li] = w0;
                ls.v[(int64_t)col * (kBW + 1) + li] = w0;
            }
            if (li == 0 && k == kBW) {
                vs[kBW] = w16;
                ls.v[(int64_t)col * (kBW + 1) + kBW] = w16;
            }
            if (li == 0) {
                bs = beta;
                ls.beta[col] = beta;
            }
        }
        __syncthreads();
        const double beta = bs;
        if (beta != 0.0) {
            const double v0 = li <= k ? vs[li] : 0.0;
            const double v16 = (li == 0 && k == kBW) ? vs[kBW] : 0.0;
            // Columns q.. of the block.
            if (q + ct < k) {
                const int cc = q + ct;
                const double h0 = h[cc][col + li];
                const double h16 = (li == 0 && k == kBW) ? h[cc][col + kBW] : 0.0;
                double sp = v0 * h0 + v16 * h16;
#pragma unroll
                for (int o = kBW / 2; o > 0; o >>= 1) sp += __shfl_xor(sp, o, kBW);
                sp *= beta;
                if (li <= k) h[cc][col + li] = h0 - sp * v0;
                if (li == 0 && k == kBW) h[cc][col + kBW] = h16 - sp * v16;
            }
            // Right-hand sides (rows q .. q + k of the staged block).
            if (ct < ka) {
                const double g0 = q + li < 2 * kBW ? gl[ct][q + li] : 0.0;
                const double g16 = (li == 0 && k == kBW) ? gl[ct][q + kBW] : 0.0;
                double sp = v0 * g0 + v16 * g16;
#pragma unroll
                for (int o = kBW / 2; o > 0; o >>= 1) sp += __shfl_xor(sp, o, kBW);
                sp *= beta;
                if (li <= k) gl[ct][q + li] = g0 - sp * v0;
                if (li == 0 && k == kBW) gl[ct][q + kBW] = g16 - sp * v16;
            }
        }
        __syncthreads();
    }
    for (int e = t; e < k * rows; e += kWG) {
        const int col = e / rows, row = e % rows;
        ls.H[(int64_t)(c0 + col) * kLdH + row] = h[col][row];
    }
    for (int e = t; e < kBW * 2 * kBW; e += kWG) {
        const int c = e / (2 * kBW), r = e % (2 * kBW);
        if (c < ka && r < 2 * k) ls.G[(int64_t)c * kLdH + c0 + r] = gl[c][r];
    }
    // Residual estimate of each right-hand side: the norm of its transformed
    // rows (j+1)k .. (j+2)k-1 (rows k .. 2k-1 of the staged block).
    if (t < ka) {
        double e2 = 0.0;
        for (int i = k; i < 2 * k; ++i) e2 += gl[t][i] * gl[t][i];
        est2[t] = e2;
    }
    __syncthreads();
    if (t == 0) {
        int conv = 1;
        for (int c = 0; c < ka; ++c) {
            const double est = sqrt(est2[c]);
            ls.est[c] = est;
            if (est > rtol * ls.rho0[c]) conv = 0;
        }
        const int f = flag[0] | (conv ? 1 : 0);
        flag[0] = f;
        flag[2] += 1;
        if (f) flag[1] = 1;
    }
}

// Y = R^{-1} G_top (R: leading J x J upper triangle of H, J = nblk * k; ka
// right-hand sides), written as nblk padded 16x16 coefficient blocks
// Cy[blk * 256 + kk * 16 + c].
__global__ __launch_bounds__(kWG) void k_bsolve(int nblk, int k, int ka, LsView ls, double* __restrict__ Cy) {
    constexpr int kStrip = 8;   // rows of H staged in LDS at a time
    __shared__ double y[kLdH][kBW];
    __shared__ double part[kBW][kBW + 1];
    __shared__ double hs[kStrip][kBlockStepsMax * kBW + 1];
    const int J = nblk * k;
    const int c = threadIdx.x & (kBW - 1), g = threadIdx.x / kBW;
    // y starts as the right-hand side G; row i is overwritten by the solution
    // once the rows below it are solved.
    for (int e = threadIdx.x; e < kLdH * kBW; e += kWG) {
        const int i = e / kBW, cc = e % kBW;
        y[i][cc] = i < J ? ls.G[(int64_t)cc * kLdH + i] : 0.0;
    }
    for (int i0 = (J - 1) / kStrip * kStrip; i0 >= 0 && J > 0; i0 -= kStrip) {
        __syncthreads();   // the previous strip is done with hs
        for (int e = threadIdx.x; e < kStrip * J; e += kWG) {
            const int q = e / kStrip, r = e % kStrip;
            hs[r][q] = i0 + r < J ? ls.H[(int64_t)q * kLdH + i0 + r] : 0.0;
        }
        __syncthreads();
        for (int i = min(J - 1, i0 + kStrip - 1); i >= i0; --i) {
            double s = 0.0;
            if (c < ka)
                for (int q = i + 1 + g; q < J; q += kBW) s += hs[i - i0][q] * y[q][c];
            part[g][c] = s;
            __syncthreads();
            if (g == 0 && c < ka) {
                double acc = y[i][c];
                for (int q = 0; q < kBW; ++q) acc -= part[q][c];
                y[i][c] = acc / hs[i - i0][i];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nblk * kPan; e += kWG) {
        const int blk = e / kPan, kk = (e % kPan) / kBW, cc = e % kBW;
        Cy[e] = (kk < k && cc < ka) ? y[blk * k + kk][cc] : 0.0;
    }
}

// Launch through the timing hook when there is one: the kernel carries the
// armed start/stop events in its own dispatch.
template <typename... KA, typename... A>
void blaunch_shm(BlockTimer* tm, int kind, double bytes, void (*k)(KA...), dim3 g, dim3 b, size_t shm,
                 hipStream_t st, A... args) {
    hipEvent_t e0, e1;
    if (tm) tm->begin(kind, bytes);
    if (tm && take_kernel_events(&e0, &e1))
        hipExtLaunchKernelGGL(k, g, b, shm, st, e0, e1, 0u, static_cast<KA>(args)...);
    else
        k<<<g, b, shm, st>>>(static_cast<KA>(args)...);
    if (tm) tm->end();
}

template <typename... KA, typename... A>
void blaunch(BlockTimer* tm, int kind, double bytes, void (*k)(KA...), dim3 g, dim3 b, hipStream_t st,
             A... args) {
    blaunch_shm(tm, kind, bytes, k, g, b, 0, st, args...);
}

constexpr int kDotGroup = 4;   // panels per workgroup of the dot kernel

}  // namespace

struct BlockWork {
    int64_t n = 0, n_pad = 0, ps = 0;
    int m = 0;
    int pw = kBW;                // panel width of the current solve (8 for k <= 8, else 16)
    double* panels = nullptr;   // (m + 1) basis panels, W, B, X
    double *part = nullptr, *C = nullptr, *Csum = nullptr;
    double *R1 = nullptr, *R = nullptr, *Rinv = nullptr, *nb2 = nullptr, *Cy = nullptr;
    double *npart = nullptr, *nsq = nullptr;
    double *lsbuf = nullptr, *S = nullptr;
    double *zpart = nullptr, *Sz = nullptr;   // deflation: Z^T W partials, E^{-1} Z^T W
    int* flag = nullptr;
    int* imap = nullptr;   // [0,16): column map; [16,32): active columns; [32,48): broken mask
    LsView ls{};
    double* V() const { return panels; }
    double* W() const { return panels + (int64_t)(m + 1) * ps; }
    double* Bp() const { return panels + (int64_t)(m + 2) * ps; }
    double* Xp() const { return panels + (int64_t)(m + 3) * ps; }
};

// Scratch of gmres_solve_block_noalloc, for callers that cannot allocate
// device memory: one array per GPU, held until the process ends.  Host code
// never passes `scratch` itself (its host-side name is not the device
// address); it uses the address looked up once per device below.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return kStatusInval;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return kStatusOk;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return kStatusDevice;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return kStatusDevice;
    g_scratch_ptr[device] = ptr;
    return kStatusOk;
}

void* static_scratch(int device, size_t* bytes) {
    *bytes = kStaticScratchBytes;
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

BlockWork* block_new() { return new (std::nothrow) BlockWork(); }
void block_delete(BlockWork* w) { delete w; }

namespace {

int64_t ls_entries() {
    return (int64_t)kLdH * kBlockStepsMax * kBW + (int64_t)kBlockStepsMax * kBW * (kBW + 1) +
           (int64_t)kBlockStepsMax * kBW + (int64_t)kLdH * kBW + 2 * kBW;
}

// Carves the block workspace for n rows and m block steps from an arena
// (sizing or real).
void block_carve(BlockWork* w, Arena& ar, int64_t n, int m) {
    w->n = n;
    w->n_pad = (n + 63) / 64 * 64;
    w->ps = w->n_pad * kBW;
    w->m = m;
    const int64_t nbmax = m + 2;
    w->panels = ar.take_n<double>((int64_t)(m + 4) * w->ps);
    w->part = ar.take_n<double>((int64_t)kDotGrid * nbmax * kPan);
    w->C = ar.take_n<double>(nbmax * kPan);
    w->Csum = ar.take_n<double>(nbmax * kPan);
    w->R1 = ar.take_n<double>(kPan);
    w->R = ar.take_n<double>(kPan);
    w->Rinv = ar.take_n<double>(kPan);
    w->nb2 = ar.take_n<double>(kBW);
    w->Cy = ar.take_n<double>((int64_t)(m + 1) * kPan);
    w->npart = ar.take_n<double>((int64_t)kNormGrid * kBW);
    w->nsq = ar.take_n<double>(kBW);
    w->lsbuf = ar.take_n<double>(ls_entries());
    w->S = ar.take_n<double>(kPan);
    w->zpart = ar.take_n<double>((int64_t)kBlockZMax * kZtChunksMax * kBW);
    w->Sz = ar.take_n<double>((int64_t)kBlockZMax * kBW);
    w->flag = ar.take_n<int>(3);
    w->imap = ar.take_n<int>(3 * kBW);
}

}  // namespace

size_t block_workspace_bytes(int64_t n, int m) {
    BlockWork w;
    Arena ar;
    ar.sizing = true;
    block_carve(&w, ar, n, m);
    return ar.peak;
}

int block_bind(BlockWork* w, void* mem, size_t bytes, hipStream_t st, int64_t n, int m) {
    Arena ar;
    ar.base = reinterpret_cast<uintptr_t>(mem);
    ar.cap = bytes;
    block_carve(w, ar, n, m);
    if (ar.short_ || (ar.base & 255) != 0) return kStatusNoMem;
    // Panel rows beyond n and columns beyond k stay zero through the solve.
    if (hipMemsetAsync(w->panels, 0, (size_t)(m + 4) * w->ps * sizeof(double), st) != hipSuccess ||
        hipMemsetAsync(w->lsbuf, 0, (size_t)ls_entries() * sizeof(double), st) != hipSuccess)
        return kStatusDevice;
    double* q = w->lsbuf;
    w->ls.H = q;
    q += (int64_t)kLdH * kBlockStepsMax * kBW;
    w->ls.v = q;
    q += (int64_t)kBlockStepsMax * kBW * (kBW + 1);
    w->ls.beta = q;
    q += (int64_t)kBlockStepsMax * kBW;
    w->ls.G = q;
    q += (int64_t)kLdH * kBW;
    w->ls.rho0 = q;
    q += kBW;
    w->ls.est = q;
    return kStatusOk;
}

namespace {

// k_bdots over nb = nv + gram blocks: ceil(nb / kDotGroup) groups of workgroups
// with the fewest slots each that hold the blocks (nb = 9: three groups of
// three).  Every slot loads a panel and issues a matrix-core step per row
// step, used or not, so unused slots cost loads and matrix-core time.
template <int PW>
void launch_dots(const BlockWork& w, BlockTimer* tm, double bytes, hipStream_t st, const double* V, int nv,
                 const double* W, int gram, const int* stop) {
    static_assert(kDotGroup == 4, "slot counts 1..4 are instantiated");
    const int nb = nv + gram;
    const int groups = (nb + kDotGroup - 1) / kDotGroup;
    const int ng = (nb + groups - 1) / groups;
    const dim3 grid(kDotGrid, groups);
    if (ng == 1)
        blaunch(tm, 5, bytes, k_bdots<1, PW>, grid, dim3(kWG), st, w.n_pad, w.ps, V, nv, W, gram, w.part, stop);
    else if (ng == 2)
        blaunch(tm, 5, bytes, k_bdots<2, PW>, grid, dim3(kWG), st, w.n_pad, w.ps, V, nv, W, gram, w.part, stop);
    else if (ng == 3)
        blaunch(tm, 5, bytes, k_bdots<3, PW>, grid, dim3(kWG), st, w.n_pad, w.ps, V, nv, W, gram, w.part, stop);
    else
        blaunch(tm, 5, bytes, k_bdots<4, PW>, grid, dim3(kWG), st, w.n_pad, w.ps, V, nv, W, gram, w.part, stop);
}

// C[0 .. nb) = P^T W (panels of V, then W itself when gram), summed.
void dots(const BlockWork& w, BlockTimer* tm, hipStream_t st, const double* V, int nv, const double* W,
          int gram, double* acc_into, int acc_blocks, int first, int diag_blk, double* nb2,
          const int* stop) {
    const int nb = nv + gram;
    const double bytes = (double)(nv + 1) * (double)w.n * w.pw * sizeof(double);   // panels and W, once
    if (w.pw == 8)
        launch_dots<8>(w, tm, bytes, st, V, nv, W, gram, stop);
    else
        launch_dots<kBW>(w, tm, bytes, st, V, nv, W, gram, stop);
    const int cnt = nb * kPan;
    k_breduce<<<(cnt + kBW - 1) / kBW, kWG, 0, st>>>(kDotGrid, cnt, w.part, w.C, acc_into, acc_blocks * kPan,
                                                     first, diag_blk, nb2, stop);
}

void gemm(const BlockWork& w, BlockTimer* tm, hipStream_t st, const double* V, int nb, const double* C,
          const double* IN, double sign, double* OUT, const int* stop) {
    const int64_t ntile = w.n_pad / kBW;
    const int grid = (int)std::min<int64_t>((ntile + 3) / 4, 8192);
    const double bytes = (double)(nb + (IN ? 1 : 0) + 1) * (double)w.n * w.pw * sizeof(double);
    const size_t shm = (size_t)nb * kPan * sizeof(double);   // the coefficient blocks
    if (w.pw == 8)
        blaunch_shm(tm, 6, bytes, k_bgemm<8>, dim3(grid), dim3(kWG), shm, st, w.n_pad, w.ps, V, nb, C, IN, sign, OUT,
                    stop);
    else
        blaunch_shm(tm, 6, bytes, k_bgemm<kBW>, dim3(grid), dim3(kWG), shm, st, w.n_pad, w.ps, V, nb, C, IN, sign,
                    OUT, stop);
}

// W -= V C (C: the first projection's coefficients in w.C), then the second
// projection's coefficients V^T W into w.C, accumulated into acc_into (as the
// dots() call without a Gram block would); one sweep over the panels.
constexpr int kFuseMax = 8;   // panels of the fused sweep (accumulators per lane)

// Workgroups of a sweep that leaves one partial per workgroup: one round of
// resident workgroups of `kernel` with shm bytes of dynamic LDS (at most
// kDotGrid, the partial-sum capacity), looked up once per device into cache.
std::mutex g_grid_mu;
int resident_grid(const void* kernel, int* cache, size_t shm = 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kDotGrid;
    std::lock_guard<std::mutex> lk(g_grid_mu);
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWG, shm) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 1;
        cache[dev] = std::min(kDotGrid, per_cu * cus);
    }
    return cache[dev];
}

template <int PW>
int fused_grid() {
    static int cache[64] = {};
    return resident_grid(reinterpret_cast<const void*>(k_bgemm_dots<kFuseMax, PW>), cache);
}

// Dynamic LDS of k_bgemm_gram for nb coefficient blocks (the wavefronts'
// accumulators reuse it), and its resident grid.
size_t gram_shm(int nb) { return (size_t)std::max(nb, kWG / kWave) * kPan * sizeof(double); }

template <int PW>
int gram_grid(int nb) {
    static int cache[kBlockStepsMax + 2][64] = {};
    const int blocks = std::max(nb, kWG / kWave);
    return resident_grid(reinterpret_cast<const void*>(k_bgemm_gram<PW>), cache[blocks], gram_shm(nb));
}

void gemm_dots(const BlockWork& w, BlockTimer* tm, hipStream_t st, const double* V, int nb, double* W,
               double* acc_into, int acc_blocks, const int* stop) {
    const double bytes = (double)(nb + 2) * (double)w.n * w.pw * sizeof(double);   // panels once, W in and out
    const int grid = w.pw == 8 ? fused_grid<8>() : fused_grid<kBW>();
    if (w.pw == 8)
        blaunch(tm, 6, bytes, k_bgemm_dots<kFuseMax, 8>, dim3(grid), dim3(kWG), st, w.n_pad, w.ps, V, nb,
                (const double*)w.C, (const double*)W, W, w.part, stop);
    else
        blaunch(tm, 6, bytes, k_bgemm_dots<kFuseMax, kBW>, dim3(grid), dim3(kWG), st, w.n_pad, w.ps, V, nb,
                (const double*)w.C, (const double*)W, W, w.part, stop);
    const int cnt = nb * kPan;
    k_breduce<<<(cnt + kBW - 1) / kBW, kWG, 0, st>>>(grid, cnt, w.part, w.C, acc_into, acc_blocks * kPan, 0,
                                                     -1, nullptr, stop);
}

// OUT = IN + sign * V C (as gemm), and OUT^T OUT summed into w.C (as the
// dots() call of OUT's Gram block alone would); one sweep.
void gemm_gram(const BlockWork& w, BlockTimer* tm, hipStream_t st, const double* V, int nb, const double* C,
               const double* IN, double sign, double* OUT, const int* stop) {
    const double bytes = (double)(nb + (IN ? 1 : 0) + 1) * (double)w.n * w.pw * sizeof(double);
    int grid;
    if (w.pw == 8) {
        grid = gram_grid<8>(nb);
        blaunch_shm(tm, 6, bytes, k_bgemm_gram<8>, dim3(grid), dim3(kWG), gram_shm(nb), st, w.n_pad, w.ps, V, nb, C,
                    IN, sign, OUT, w.part, stop);
    } else {
        grid = gram_grid<kBW>(nb);
        blaunch_shm(tm, 6, bytes, k_bgemm_gram<kBW>, dim3(grid), dim3(kWG), gram_shm(nb), st, w.n_pad, w.ps, V, nb,
                    C, IN, sign, OUT, w.part, stop);
    }
    k_breduce<<<kPan / kBW, kWG, 0, st>>>(grid, kPan, w.part, w.C, nullptr, 0, 0, -1, nullptr, stop);
}

// Cholesky QR applied twice to the panel `src` into `dst` (may alias):
// dst R = src, R = R2 R1 (into w.R).  test: breakdown test of the first pass
// against nb2 (NULL: the Gram diagonal).  gram_ready: w.C already holds
// src^T src (the sweep that wrote src formed it).
void cholqr2(const BlockWork& w, BlockTimer* tm, hipStream_t st, int k, const double* src, double* dst,
             int test, const double* nb2, const int* stop, bool gram_ready = false) {
    if (!gram_ready) dots(w, tm, st, nullptr, 0, src, 1, nullptr, 0, 0, -1, nullptr, stop);
    k_bchol<<<1, kWave, 0, st>>>(k, w.C, nb2, test, nullptr, w.R1, w.Rinv, w.flag, w.imap + 2 * kBW, stop);
    gemm_gram(w, tm, st, src, 1, w.Rinv, nullptr, 1.0, dst, stop);   // and dst^T dst into w.C
    k_bchol<<<1, kWave, 0, st>>>(k, w.C, nullptr, 0, w.R1, w.R, w.Rinv, w.flag, nullptr, stop);
    gemm(w, tm, st, dst, 1, w.Rinv, nullptr, 1.0, dst, stop);
}

// Residual panel W = B - A X and the column norms on the host.
// Algorithmic bytes of one SpMM: A (8-byte values, 4-byte indices, row
// pointers), the input panel (one line per row), the output panel (and B).
double spmm_bytes(const BlockWork& w, const BlockArgs& a, int mode) {
    return 12.0 * (double)a.nnz + 4.0 * (double)(w.n + 1) + (2.0 + mode) * (double)w.n * w.pw * sizeof(double);
}

// Y = A X (mode 0) or Y = B - A X with column partial sums of squares
// (mode 1), the instance for the solve's panel width.
void spmm(const BlockWork& w, const BlockArgs& a, int mode, dim3 grid, hipStream_t st, const double* X,
          const double* B, double* Y, double* part, const int* stop) {
    const double bytes = spmm_bytes(w, a, mode);
    if (mode == 0 && w.pw == 8)
        blaunch(a.timer, 7, bytes, k_bspmm<0, 8>, grid, dim3(kWG), st, w.n, a.rowptr, a.colind, a.vals, X, B, Y,
                part, stop);
    else if (mode == 0)
        blaunch(a.timer, 7, bytes, k_bspmm<0, kBW>, grid, dim3(kWG), st, w.n, a.rowptr, a.colind, a.vals, X, B, Y,
                part, stop);
    else if (w.pw == 8)
        blaunch(a.timer, 7, bytes, k_bspmm<1, 8>, grid, dim3(kWG), st, w.n, a.rowptr, a.colind, a.vals, X, B, Y,
                part, stop);
    else
        blaunch(a.timer, 7, bytes, k_bspmm<1, kBW>, grid, dim3(kWG), st, w.n, a.rowptr, a.colind, a.vals, X, B, Y,
                part, stop);
}

// S = E^{-1} Z^T P into w.Sz (deflation basis of a).
void coarse(const BlockWork& w, const BlockArgs& a, const double* P, const int* stop) {
    // About 256 entries of Z^T per workgroup (Z's rows are shared out over
    // its columns), at most kZtChunksMax workgroups per column.
    const int nch = (int)std::max<int64_t>(1, std::min<int64_t>(kZtChunksMax, (w.n + 256LL * a.R - 1) / (256LL * a.R)));
    if (w.pw == 8)
        k_bzt<8><<<dim3((unsigned)a.R, (unsigned)nch), kWG, 0, a.st>>>(nch, a.ztrp, a.ztci, a.ztv, P, w.zpart, stop);
    else
        k_bzt<kBW><<<dim3((unsigned)a.R, (unsigned)nch), kWG, 0, a.st>>>(nch, a.ztrp, a.ztci, a.ztv, P, w.zpart,
                                                                        stop);
    k_bcoarse<<<1, kWG, 0, a.st>>>(a.R, nch, w.zpart, a.Einv, w.Sz, stop);
}

// P += sign * M S (k_bzapply, S in w.Sz): pw lanes per row, kWG / pw rows per
// workgroup and round, 4096 workgroups at most.
void zapply(const BlockWork& w, hipStream_t st, int R, const int* mrp, const int* mci, const double* mv,
            double sign, double* P, const int* stop) {
    const int rpr = kWG / w.pw;
    const unsigned g = (unsigned)std::min<int64_t>((w.n + rpr - 1) / rpr, 4096);
    if (w.pw == 8)
        k_bzapply<8><<<g, kWG, 0, st>>>(w.n, R, mrp, mci, mv, w.Sz, sign, P, stop);
    else
        k_bzapply<kBW><<<g, kWG, 0, st>>>(w.n, R, mrp, mci, mv, w.Sz, sign, P, stop);
}

// W = P W = W - A Z E^{-1} Z^T W (no-op without a deflation basis).
void project(const BlockWork& w, const BlockArgs& a, double* W, const int* stop) {
    if (a.R == 0) return;
    coarse(w, a, W, stop);
    zapply(w, a.st, a.R, a.azrp, a.azci, a.azv, -1.0, W, stop);
}

// W = B - A X, h_raw[c] = ||w_c||; then W = P W and h_nrm[c] = ||P w_c||
// (h_nrm = h_raw without a deflation basis).
int residual(const BlockWork& w, const BlockArgs& a, double* h_raw, double* h_nrm) {
    spmm(w, a, 1, dim3(kNormGrid), a.st, (const double*)w.Xp(), (const double*)w.Bp(), w.W(), w.npart, nullptr);
    k_bcolsum<<<1, kWG, 0, a.st>>>(kNormGrid, w.npart, w.nsq);
    double sq[kBW], sp[kBW];
    if (hipMemcpyAsync(sq, w.nsq, sizeof(sq), hipMemcpyDeviceToHost, a.st) != hipSuccess) return kStatusDevice;
    if (a.R > 0) {
        project(w, a, w.W(), nullptr);
        k_bnorm<<<kNormGrid, kWG, 0, a.st>>>(w.n, w.pw, w.W(), w.npart);
        k_bcolsum<<<1, kWG, 0, a.st>>>(kNormGrid, w.npart, w.nsq);
        if (hipMemcpyAsync(sp, w.nsq, sizeof(sp), hipMemcpyDeviceToHost, a.st) != hipSuccess)
            return kStatusDevice;
    }
    if (hipStreamSynchronize(a.st) != hipSuccess) return kStatusDevice;
    for (int c = 0; c < kBW; ++c) {
        h_raw[c] = std::sqrt(sq[c]);
        h_nrm[c] = a.R > 0 ? std::sqrt(sp[c]) : h_raw[c];
    }
    return kStatusOk;
}


}  // namespace

int block_solve(BlockWork* w, const BlockArgs& a, BlockResult* res) {
    const hipStream_t st = a.st;
    const int k = a.k, m = a.m;
    *res = BlockResult{};
    // Panels of 8 columns for up to 8 right-hand sides (half the bytes of
    // the 16-wide rows), else 16; both fit the workspace carved for 16.
    w->pw = k <= 8 ? 8 : kBW;
    w->ps = w->n_pad * w->pw;
    const int64_t pe = w->n * w->pw;
    const unsigned gpe = (unsigned)((pe + kWG - 1) / kWG);
    k_bpack<<<gpe, kWG, 0, st>>>(w->n, k, w->pw, a.B, w->Bp());
    k_bpack<<<gpe, kWG, 0, st>>>(w->n, k, w->pw, a.X0, w->Xp());
    // rho0_c = ||b_c - A x0_c|| (unprojected); the tests use ||P (b_c - A x_c)||.
    double rho0[kBW], rn[kBW], raw[kBW];
    int s = residual(*w, a, rho0, rn);
    if (s != kStatusOk) return s;
    double rho_max = 0.0;
    for (int c = 0; c < k; ++c) {
        if (!(rho0[c] > 0.0)) return kStatusInval;   // zero (or non-finite) initial residual column
        rho_max = std::max(rho_max, rho0[c]);
    }
    res->rho0 = rho_max;
    int64_t steps = 0;
    int cycles = 0, status = kStatusMaxIter;
    double est_max = 1.0;
    for (;;) {
        // Active columns: residual not yet below rtol * rho0_c.
        int act[kBW], ka = 0;
        for (int c = 0; c < k; ++c)
            if (rn[c] > a.rtol * rho0[c]) act[ka++] = c;
        if (ka == 0) {
            status = kStatusOk;
            break;
        }
        if (steps >= a.max_steps) {
            status = kStatusMaxIter;
            break;
        }
        // Starting block from the active residual columns: V_0 S = R.
        int hmap[3 * kBW];
        for (int c = 0; c < kBW; ++c) {
            hmap[c] = c < ka ? act[c] : -1;
            hmap[kBW + c] = c < ka ? act[c] : 0;
        }
        if (hipMemcpyAsync(w->imap, hmap, 2 * kBW * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemsetAsync(w->flag, 0, sizeof(int), st) != hipSuccess ||
            hipMemsetAsync(w->imap + 2 * kBW, 0, kBW * sizeof(int), st) != hipSuccess)
            return kStatusDevice;
        k_bselect<<<gpe, kWG, 0, st>>>(w->n, w->pw, w->imap, w->W());
        cholqr2(*w, a.timer, st, ka, w->W(), w->V(), 1, nullptr, nullptr);
        // A residual column dependent on the earlier ones adds no basis
        // vector: keep kb independent columns, S = their rows of R (kb x ka).
        double hR[kPan];
        if (hipMemcpyAsync(hR, w->R, sizeof(hR), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hmap + 2 * kBW, w->imap + 2 * kBW, kBW * sizeof(int), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return kStatusDevice;
        int indep[kBW], kb = 0;
        for (int c = 0; c < ka; ++c)
            if (!hmap[2 * kBW + c]) indep[kb++] = c;
        double hS[kPan] = {};
        for (int q = 0; q < kb; ++q)
            for (int c = 0; c < ka; ++c) hS[q * kBW + c] = hR[indep[q] * kBW + c];
        double r0a[kBW] = {};
        for (int c = 0; c < ka; ++c) r0a[c] = rho0[act[c]];
        if (hipMemcpyAsync(w->S, hS, sizeof(hS), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(w->ls.rho0, r0a, sizeof(r0a), hipMemcpyHostToDevice, st) != hipSuccess)
            return kStatusDevice;
        if (kb < ka) {
            int cmap[kBW];
            for (int c = 0; c < kBW; ++c) cmap[c] = c < kb ? indep[c] : -1;
            if (hipMemcpyAsync(w->imap, cmap, kBW * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess)
                return kStatusDevice;
            k_bselect<<<gpe, kWG, 0, st>>>(w->n, w->pw, w->imap, w->V());
        }
        // flag[0]: breakdown / convergence bits, flag[1]: the cycle has
        // ended (gate of its later kernels), flag[2]: steps done.  The
        // cycle's steps are enqueued without waiting for the host; the steps
        // after the one that ends the cycle return at once.
        if (hipMemsetAsync(w->flag, 0, 3 * sizeof(int), st) != hipSuccess) return kStatusDevice;
        k_bls_init<<<1, kWG, 0, st>>>(kb, ka, w->S, w->ls);
        ++cycles;
        const int* stop = w->flag + 1;
        const int nst = (int)std::min<int64_t>(m, a.max_steps - steps);
        for (int j = 0; j < nst; ++j) {
            if (a.timer) a.timer->step(j);
            double* Vj = w->V() + (int64_t)j * w->ps;
            double* Vn = w->V() + (int64_t)(j + 1) * w->ps;
            const unsigned g16 = (unsigned)((w->n + kWG / w->pw - 1) / (kWG / w->pw));
            spmm(*w, a, 0, dim3(g16), st, (const double*)Vj, nullptr, w->W(), nullptr, stop);
            project(*w, a, w->W(), stop);   // W = P A V_j
            // BCGS2: two projections onto V_0..V_j; the first also gives the
            // squared column norms of A V_j (the breakdown reference).
            dots(*w, a.timer, st, w->V(), j + 1, w->W(), 1, w->Csum, j + 1, 1, j + 1, w->nb2, stop);
            if (j + 1 <= kFuseMax) {
                // First projection and second dot pass in one sweep.
                gemm_dots(*w, a.timer, st, w->V(), j + 1, w->W(), w->Csum, j + 1, stop);
            } else {
                gemm(*w, a.timer, st, w->V(), j + 1, w->C, w->W(), -1.0, w->W(), stop);
                dots(*w, a.timer, st, w->V(), j + 1, w->W(), 0, w->Csum, j + 1, 0, -1, nullptr, stop);
            }
            // Second projection; its sweep also forms W^T W for the CholQR.
            gemm_gram(*w, a.timer, st, w->V(), j + 1, w->C, w->W(), -1.0, w->W(), stop);
            cholqr2(*w, a.timer, st, kb, w->W(), Vn, 1, w->nb2, stop, true);
            k_bls<<<1, kWG, 0, st>>>(j, kb, ka, a.rtol, w->Csum, w->R, w->ls, w->flag);
        }
        double est[kBW];
        int hf[3] = {0, 0, 0};
        if (hipMemcpyAsync(est, w->ls.est, sizeof(est), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hf, w->flag, sizeof(hf), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return kStatusDevice;
        const int jd = hf[2];
        steps += jd;
        if (a.timer) a.timer->cycle_done(jd);
        est_max = 0.0;
        for (int c = 0; c < ka; ++c) est_max = std::max(est_max, est[c] / r0a[c]);
        // X[:, act] += V Y (through the free W panel).
        k_bsolve<<<1, kWG, 0, st>>>(jd, kb, ka, w->ls, w->Cy);
        gemm(*w, a.timer, st, w->V(), jd, w->Cy, nullptr, 1.0, w->W(), nullptr);
        k_bscatter<<<gpe, kWG, 0, st>>>(w->n, w->pw, ka, w->imap + kBW, w->W(), w->Xp());
        if ((s = residual(*w, a, raw, rn)) != kStatusOk) return s;
        for (int c = 0; c < k; ++c)
            if (!std::isfinite(rn[c])) return kStatusNonFinite;
    }
    if (a.R > 0) {
        // x_c = x_hat_c + Z E^{-1} Z^T (b_c - A x_hat_c) (eq. precond2); the
        // true residuals are then recomputed.
        spmm(*w, a, 1, dim3(kNormGrid), st, (const double*)w->Xp(), (const double*)w->Bp(), w->W(), w->npart,
             nullptr);
        coarse(*w, a, w->W(), nullptr);
        zapply(*w, st, a.R, a.zrp, a.zci, a.zv, 1.0, w->Xp(), nullptr);
        if ((s = residual(*w, a, raw, rn)) != kStatusOk) return s;
        for (int c = 0; c < k; ++c) rn[c] = raw[c];
    }
    const int64_t ue = w->n * k;
    k_bunpack<<<(unsigned)((ue + kWG - 1) / kWG), kWG, 0, st>>>(w->n, k, w->pw, w->Xp(), a.X);
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusDevice;
    double tr = 0.0;
    for (int c = 0; c < k; ++c) tr = std::max(tr, rn[c] / rho0[c]);
    res->steps = steps;
    res->cycles = cycles;
    res->status = status;
    res->rel_res_est = est_max;
    res->rel_res_true = tr;
    return kStatusOk;
}

GM_DEBUG_ACCESSOR(dbg_take_block)

}  // namespace gm
