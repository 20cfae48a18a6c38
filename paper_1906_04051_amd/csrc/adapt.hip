// Adaptive spectral deflation (arXiv 1906.04051, Sec. 3.3): GMRES(m) on the
// right-preconditioned operator A M^{-1} (eq. precond1) with
//   M^{-1} = I + U (|mu| T^{-1} - I) U^T      (eq. precond2),  T = U^T A U (eq. tau_mat),
// U orthonormal, N x r, r <= r_max.  At every restart one Ritz vector of the
// cycle's Hessenberg matrix H_k for its smallest eigenvalue (inverse
// iteration) gives u = V_k z (eq. precond3), which is orthonormalised against
// U and appended (A u to AU, T extended); beyond r_max the direction of U
// belonging to the largest eigenvalue of T is removed by a Householder
// rotation of U, AU and T.  |mu| comes from power iteration on H_k.
//
// Per Arnoldi step the operator is applied as
//   s = C (U^T x),  C = |mu| T^{-1} - I   (dot kernel + one small kernel),
//   y = A x + (A U) s                      (SpMV, then the dense correction),
// and a cycle ends with x += M^{-1} (V_k y_k), so M may change between cycles.
// The device state (r, |mu|, flags) lives in AdaptState, so a whole cycle is
// enqueued (and captured) without the host knowing r.
//
// Fixed constants shared with the reference solution: 30 power iterations,
// 20 inverse iterations, both from the normalised ones vector; append only
// when ||u|| > 1e-8 after two Gram-Schmidt passes; singular H_k or T detected
// as |pivot| <= k eps max|entries| (then no append, or C = 0).
#include "internal.hpp"

namespace gm {

constexpr int kAJ = kAdaptMax + 2;   // columns a dot kernel handles (basis + one extra)
constexpr int kKP = 30;              // power iterations
constexpr int kKI = 20;              // inverse iterations
constexpr int kSW = 64;              // threads of the small dense kernels (one wavefront)

// ------------------------------------------------------------ dot products
// Partial sums over this workgroup's rows of B_q . (scale * x) for the first
// nb columns of B (nb = st->r when use_r, else 0) and, when xtra is given, of
// xtra . (scale * x) in slot nb.  part[slot * NB + block], fixed order.
// Vectors are zero padded to whole 2-row tiles.
// Column loads of the dot and update kernels: plain, or with the
// non-temporal hint (NT) for the per-step operator when U and A U outgrow
// the last-level cache: they are read once per step, while the leading
// Krylov columns and the matrix kept there are read again every step.
template <bool NT>
__device__ __forceinline__ double2 ld_col2(const double* p) {
    if constexpr (NT) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v t = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
        return make_double2(t.x, t.y);
    } else {
        return *reinterpret_cast<const double2*>(p);
    }
}

template <bool NT>
__global__ __launch_bounds__(kWG) void k_udots(int n, int64_t ldv, const double* __restrict__ B,
                                               const AdaptState* __restrict__ st, int use_r,
                                               const double* __restrict__ xtra,
                                               const double* __restrict__ x,
                                               const double* __restrict__ xscale,
                                               double* __restrict__ part, int NB, const Ctrl* ctrl,
                                               int gate) {
    __shared__ double red[kWG / kWave][kAJ];
    const int nb = use_r ? st->r : 0;
    const int ns = nb + (xtra ? 1 : 0);
    const double sc = xscale ? *xscale : 1.0;
    if (gated(ctrl, gate) || ns == 0) return;
    double acc[kAJ];
#pragma unroll
    for (int q = 0; q < kAJ; ++q) acc[q] = 0;
    const int64_t stride = (int64_t)gridDim.x * kWG * 2;
    for (int64_t i0 = ((int64_t)blockIdx.x * kWG + threadIdx.x) * 2; i0 < n; i0 += stride) {
        const double2 xv = *reinterpret_cast<const double2*>(x + i0);
        const double x0 = xv.x * sc, x1 = xv.y * sc;
        double2 bv[kAJ];
#pragma unroll
        for (int q = 0; q < kAJ; ++q)
            if (q < ns) bv[q] = ld_col2<NT>((q < nb ? B + q * ldv : xtra) + i0);
#pragma unroll
        for (int q = 0; q < kAJ; ++q)
            if (q < ns) acc[q] += bv[q].x * x0 + bv[q].y * x1;
    }
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int q = 0; q < kAJ; ++q) {
        if (q < ns) {
            const double t = wave_sum(acc[q]);
            if (ln == 0) red[wv][q] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < ns) {
        double t = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWG / kWave; ++w) t += red[w][threadIdx.x];
        part[(int64_t)threadIdx.x * NB + blockIdx.x] = t;
    }
}

// t_q = sum of the partials of slot q (q < ns, fixed order: lane-strided
// sums, then the wave butterfly; one wavefront per slot); then
//   C given: s = C t over the first nb slots (C row-major, leading dim ldc),
//   else     s = t.
// tsave (optional) receives t.
constexpr int kUC = 1024;   // threads of k_ucoef (16 wavefronts)

__global__ __launch_bounds__(kUC) void k_ucoef(const AdaptState* __restrict__ st, int use_r,
                                               int has_xtra, const double* __restrict__ part,
                                               int NB, const double* __restrict__ C, int ldc,
                                               double* __restrict__ s, double* __restrict__ tsave,
                                               const Ctrl* ctrl, int gate) {
    __shared__ double t[kAJ];
    const int nb = use_r ? st->r : 0;
    const int ns = nb + (has_xtra ? 1 : 0);
    if (gated(ctrl, gate) || ns == 0) return;
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
    for (int q = wv; q < ns; q += kUC / kWave) {
        double acc = 0;
        for (int b = ln; b < NB; b += kWave) acc += part[(int64_t)q * NB + b];
        acc = wave_sum(acc);
        if (ln == 0) t[q] = acc;
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < ns) {
        if (tsave) tsave[i] = t[i];
        if (C) {
            if (i < nb) {
                double v = 0;
                for (int q = 0; q < nb; ++q) v += C[(int64_t)i * ldc + q] * t[q];
                s[i] = v;
            }
        } else {
            s[i] = t[i];
        }
    }
}

// y += sign * sum_{q < r} B_q s_q  (B = A U for the operator, U for
// Gram-Schmidt updates), two rows per thread.
template <bool NT>
__global__ __launch_bounds__(kWG) void k_ucorr(int n, int64_t ldv, const double* __restrict__ B,
                                               const AdaptState* __restrict__ st,
                                               const double* __restrict__ s, double sign,
                                               double* __restrict__ y, const Ctrl* ctrl, int gate) {
    __shared__ double sl[kAJ];
    const int nb = st->r;
    if (gated(ctrl, gate) || nb == 0) return;
    if (threadIdx.x < nb) sl[threadIdx.x] = sign * s[threadIdx.x];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWG * 2;
    for (int64_t i0 = ((int64_t)blockIdx.x * kWG + threadIdx.x) * 2; i0 < n; i0 += stride) {
        double2 bv[kAJ];
#pragma unroll
        for (int q = 0; q < kAJ; ++q)
            if (q < nb) bv[q] = ld_col2<NT>(B + q * ldv + i0);
        double2 yv = *reinterpret_cast<const double2*>(y + i0);
#pragma unroll
        for (int q = 0; q < kAJ; ++q)
            if (q < nb) {
                yv.x += bv[q].x * sl[q];
                yv.y += bv[q].y * sl[q];
            }
        *reinterpret_cast<double2*>(y + i0) = yv;
    }
}

// x += d + sum_{q < r} U_q s_q   (x += M^{-1} d once s = C U^T d).
__global__ __launch_bounds__(kWG) void k_uaxpy(int n, int64_t ldv, const double* __restrict__ U,
                                               const AdaptState* __restrict__ st,
                                               const double* __restrict__ s,
                                               const double* __restrict__ d,
                                               double* __restrict__ x, const Ctrl* ctrl, int gate) {
    __shared__ double sl[kAJ];
    const int nb = st->r;
    if (gated(ctrl, gate)) return;
    if (threadIdx.x < nb) sl[threadIdx.x] = s[threadIdx.x];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        double v = d[i];
        for (int q = 0; q < nb; ++q) v += U[q * ldv + i] * sl[q];
        x[i] += v;
    }
}

// out = sum_{q < k} V_q coef_q with k = ctrl->k (the cycle's basis size).
__global__ __launch_bounds__(kWG) void k_vcomb(int n, int64_t ldv, const double* __restrict__ V,
                                               const double* __restrict__ coef,
                                               double* __restrict__ out, const Ctrl* ctrl,
                                               int gate) {
    __shared__ double c_l[kMaxM];
    if (gated(ctrl, gate)) return;
    const int k = ctrl->k;
    for (int t = threadIdx.x; t < k; t += kWG) c_l[t] = coef[t];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        double acc = 0;
        for (int q = 0; q < k; ++q) acc += V[q * ldv + i] * c_l[q];
        out[i] = acc;
    }
}

// ----------------------------------------------------- small dense kernels
// Work on k x k row-major matrices in LDS with one wavefront (kSW threads,
// rows i = lane, lane + kSW, ...).

__device__ __forceinline__ double sw_sum(double v) { return wave_sum(v); }

// z <- KP power iterations on M (k x k) from ones/sqrt(k); returns ||M z||.
__device__ double sw_power(int k, const double* M, double* z, double* z2) {
    const int ln = threadIdx.x;
    for (int i = ln; i < k; i += kSW) z[i] = 1.0 / sqrt((double)k);
    __syncthreads();
    for (int it = 0; it < kKP; ++it) {
        double ss = 0;
        for (int i = ln; i < k; i += kSW) {
            double v = 0;
            for (int q = 0; q < k; ++q) v += M[i * k + q] * z[q];
            z2[i] = v;
            ss += v * v;
        }
        const double nz = sqrt(sw_sum(ss));
        __syncthreads();
        if (nz == 0.0) return 0.0;
        for (int i = ln; i < k; i += kSW) z[i] = z2[i] / nz;
        __syncthreads();
    }
    double ss = 0;
    for (int i = ln; i < k; i += kSW) {
        double v = 0;
        for (int q = 0; q < k; ++q) v += M[i * k + q] * z[q];
        ss += v * v;
    }
    return sqrt(sw_sum(ss));
}

// In-place LU with partial pivoting (first row of largest |entry| in the
// column); false when |pivot| <= k eps max|M|.
__device__ bool sw_lu(int k, double* M, int* piv) {
    const int ln = threadIdx.x;
    double mx = 0;
    for (int e = ln; e < k * k; e += kSW) mx = fmax(mx, fabs(M[e]));
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
    const double tiny = (double)k * 2.220446049250313e-16 * mx;
    for (int p = 0; p < k; ++p) {
        // argmax |M[i][p]| over i >= p, smallest index among equals
        double bv = -1.0;
        int bi = k;
        for (int i = p + ln; i < k; i += kSW) {
            const double v = fabs(M[i * k + p]);
            if (v > bv) { bv = v; bi = i; }
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, kWave);
            const int oi = __shfl_xor(bi, o, kWave);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (ln == 0) piv[p] = bi;
        if (!(bv > tiny)) {
            __syncthreads();
            return false;
        }
        if (bi != p)
            for (int q = ln; q < k; q += kSW) {
                const double t = M[p * k + q];
                M[p * k + q] = M[bi * k + q];
                M[bi * k + q] = t;
            }
        __syncthreads();
        const double d = M[p * k + p];
        for (int i = p + 1 + ln; i < k; i += kSW) M[i * k + p] /= d;
        __syncthreads();
        for (int e = ln; e < (k - p - 1) * (k - p - 1); e += kSW) {
            const int i = p + 1 + e / (k - p - 1), q = p + 1 + e % (k - p - 1);
            M[i * k + q] -= M[i * k + p] * M[p * k + q];
        }
        __syncthreads();
    }
    return true;
}

// z <- (P L U)^{-1} z: row swaps, unit lower L, then U (column oriented).
__device__ void sw_lu_solve(int k, const double* LU, const int* piv, double* z) {
    const int ln = threadIdx.x;
    if (ln == 0)
        for (int p = 0; p < k; ++p) {
            const int q = piv[p];
            if (q != p) {
                const double t = z[p];
                z[p] = z[q];
                z[q] = t;
            }
        }
    __syncthreads();
    for (int p = 0; p < k; ++p) {
        const double zp = z[p];
        for (int i = p + 1 + ln; i < k; i += kSW) z[i] -= LU[i * k + p] * zp;
        __syncthreads();
    }
    for (int p = k - 1; p >= 0; --p) {
        if (ln == 0) z[p] /= LU[p * k + p];
        __syncthreads();
        const double zp = z[p];
        for (int i = ln; i < p; i += kSW) z[i] -= LU[i * k + p] * zp;
        __syncthreads();
    }
}

// Ritz step of one restart: |mu| by power iteration on H_k, the eigenvector
// of H_k's smallest eigenvalue by inverse iteration; zc = z_i * vscale[i]
// (coefficients on the stored basis).  st->ok = 0 when H_k is singular.
__global__ __launch_bounds__(kSW) void k_ritz(int m, const double* __restrict__ Hraw,
                                              const double* __restrict__ vscale,
                                              AdaptState* __restrict__ st,
                                              double* __restrict__ zc, const Ctrl* ctrl, int gate) {
    __shared__ double H[kMaxM * kMaxM];
    __shared__ double z[kMaxM], z2[kMaxM];
    __shared__ int piv[kMaxM];
    if (gated(ctrl, gate)) return;
    const int k = ctrl->k;
    const int ln = threadIdx.x;
    if (k < 1) {
        if (ln == 0) st->ok = 0;
        return;
    }
    // Only the Hessenberg band (rows i <= q + 1 of column q) is ever written;
    // the entries below it are zero by definition, not read from memory.
    for (int e = ln; e < k * k; e += kSW) {
        const int i = e / k, q = e % k;
        H[e] = (i <= q + 1) ? Hraw[(int64_t)i * m + q] : 0.0;
    }
    __syncthreads();
    const double mu = sw_power(k, H, z, z2);
    __syncthreads();
    const bool ok = sw_lu(k, H, piv);
    if (ok) {
        for (int i = ln; i < k; i += kSW) z[i] = 1.0 / sqrt((double)k);
        __syncthreads();
        for (int it = 0; it < kKI; ++it) {
            sw_lu_solve(k, H, piv, z);
            double ss = 0;
            for (int i = ln; i < k; i += kSW) ss += z[i] * z[i];
            const double nz = sqrt(sw_sum(ss));
            __syncthreads();
            for (int i = ln; i < k; i += kSW) z[i] /= nz;
            __syncthreads();
        }
        for (int i = ln; i < k; i += kSW) zc[i] = z[i] * vscale[i];
    }
    if (ln == 0) {
        st->mu = mu;
        st->ok = ok ? 1 : 0;
    }
}

// ||u||: slot 0 of the partials; the candidate is kept when ||u|| > 1e-8.
__global__ __launch_bounds__(kWG) void k_unorm(const double* __restrict__ part, int NB,
                                               AdaptState* __restrict__ st, const Ctrl* ctrl,
                                               int gate) {
    __shared__ double red[kWG / kWave];
    if (gated(ctrl, gate)) return;
    double acc = 0;
    for (int b = threadIdx.x; b < NB; b += kWG) acc += part[b];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) {
        const double nu = sqrt(acc);
        st->nu = nu;
        if (!(nu > 1e-8)) st->ok = 0;
    }
}

// u *= 1 / ||u|| for an accepted candidate.
__global__ __launch_bounds__(kWG) void k_uscale(int n, double* __restrict__ u,
                                                const AdaptState* __restrict__ st, const Ctrl* ctrl,
                                                int gate) {
    if (gated(ctrl, gate) || !st->ok) return;
    const double inv = 1.0 / st->nu;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) u[i] *= inv;
}

// T update of one restart (one wavefront): append the new row / column
// (tcol[q] = U_q . A u for q < r and u . A u at q = r; trow[q] = u . A U_q),
// remove the direction of T's largest eigenvalue beyond r_max (Householder
// vector to hvec), and form C = |mu| T^{-1} - I (zero when T is singular).
// T and C are row-major with leading dimension ld = r_max + 1.
__global__ __launch_bounds__(kSW) void k_tupdate(int rmax, double* __restrict__ T,
                                                 double* __restrict__ C,
                                                 const double* __restrict__ tcol,
                                                 const double* __restrict__ trow,
                                                 double* __restrict__ hvec,
                                                 AdaptState* __restrict__ st, const Ctrl* ctrl,
                                                 int gate) {
    __shared__ double M[(kAdaptMax + 1) * (kAdaptMax + 1)];
    __shared__ double LU[(kAdaptMax + 1) * (kAdaptMax + 1)];
    __shared__ double z[kAdaptMax + 1], z2[kAdaptMax + 1], h[kAdaptMax + 1];
    __shared__ int piv[kAdaptMax + 1];
    if (gated(ctrl, gate)) return;
    const int ld = rmax + 1;
    const int ln = threadIdx.x;
    const int r = st->r;
    const int ok = st->ok;
    if (ok) {
        for (int q = ln; q <= r; q += kSW) T[q * ld + r] = tcol[q];
        for (int q = ln; q < r; q += kSW) T[r * ld + q] = trow[q];
    }
    __syncthreads();   // the new row / column is read back below by other lanes
    int rr = r + (ok ? 1 : 0);
    for (int e = ln; e < rr * rr; e += kSW) M[e] = T[(e / rr) * ld + e % rr];
    __syncthreads();
    const int remove = rr > rmax;
    if (remove) {
        sw_power(rr, M, z, z2);
        double ss = 0;
        for (int i = ln; i < rr; i += kSW) ss += z[i] * z[i];
        const double nw = sqrt(sw_sum(ss));
        const double alpha = (z[0] >= 0.0) ? -nw : nw;
        for (int i = ln; i < rr; i += kSW) h[i] = z[i] - (i == 0 ? alpha : 0.0);
        __syncthreads();
        double hh = 0;
        for (int i = ln; i < rr; i += kSW) hh += h[i] * h[i];
        const double nh = sqrt(sw_sum(hh));
        __syncthreads();
        for (int i = ln; i < rr; i += kSW) {
            h[i] /= nh;
            hvec[i] = h[i];
        }
        __syncthreads();
        // M <- M Q (rows), then Q M (columns), Q = I - 2 h h^T.
        for (int i = ln; i < rr; i += kSW) {
            double p = 0;
            for (int q = 0; q < rr; ++q) p += M[i * rr + q] * h[q];
            for (int q = 0; q < rr; ++q) M[i * rr + q] -= 2.0 * p * h[q];
        }
        __syncthreads();
        for (int q = ln; q < rr; q += kSW) {
            double p = 0;
            for (int i = 0; i < rr; ++i) p += h[i] * M[i * rr + q];
            for (int i = 0; i < rr; ++i) M[i * rr + q] -= 2.0 * h[i] * p;
        }
        __syncthreads();
        // Drop row and column 0.
        for (int e = ln; e < (rr - 1) * (rr - 1); e += kSW) {
            const int i = e / (rr - 1), q = e % (rr - 1);
            T[i * ld + q] = M[(i + 1) * rr + (q + 1)];
        }
        __syncthreads();
        rr -= 1;
        for (int e = ln; e < rr * rr; e += kSW) M[e] = T[(e / rr) * ld + e % rr];
        __syncthreads();
    }
    // C = |mu| T^{-1} - I, column by column through the LU of T.
    for (int e = ln; e < rr * rr; e += kSW) LU[e] = M[e];
    __syncthreads();
    const bool nonsing = rr > 0 && sw_lu(rr, LU, piv);
    const double mu = st->mu;
    for (int q = 0; q < rr; ++q) {
        if (nonsing) {
            for (int i = ln; i < rr; i += kSW) z[i] = (i == q) ? 1.0 : 0.0;
            __syncthreads();
            sw_lu_solve(rr, LU, piv, z);
            for (int i = ln; i < rr; i += kSW) C[i * ld + q] = mu * z[i] - (i == q ? 1.0 : 0.0);
        } else {
            for (int i = ln; i < rr; i += kSW) C[i * ld + q] = 0.0;
        }
        __syncthreads();
    }
    if (ln == 0) {
        st->r_old = r;
        st->r_new = rr;
        st->remove = remove;
    }
}

// Commits an accepted candidate: U[:, r_old] = u, AU[:, r_old] = A u.
__global__ __launch_bounds__(kWG) void k_ucommit(int64_t ldv, double* __restrict__ U,
                                                 double* __restrict__ AU,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ au,
                                                 const AdaptState* __restrict__ st,
                                                 const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate) || !st->ok) return;
    const int c = st->r_old;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < ldv; i += stride) {
        U[c * ldv + i] = u[i];
        AU[c * ldv + i] = au[i];
    }
}

// Removal: U <- (U Q)[:, 1:], AU <- (AU Q)[:, 1:] with Q = I - 2 h h^T over
// the nc = r_old + ok columns; rows are independent, so it runs in place.
__global__ __launch_bounds__(kWG) void k_householder(int n, int64_t ldv, double* __restrict__ U,
                                                     double* __restrict__ AU,
                                                     const double* __restrict__ hvec,
                                                     const AdaptState* __restrict__ st,
                                                     const Ctrl* ctrl, int gate) {
    __shared__ double hl[kAJ];
    if (gated(ctrl, gate) || !st->remove) return;
    const int nc = st->r_old + st->ok;
    if (threadIdx.x < nc) hl[threadIdx.x] = hvec[threadIdx.x];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        for (int mi = 0; mi < 2; ++mi) {
            double* Mx = mi == 0 ? U : AU;
            double v[kAJ];
            double p = 0;
#pragma unroll
            for (int q = 0; q < kAJ; ++q)
                if (q < nc) {
                    v[q] = Mx[q * ldv + i];
                    p += v[q] * hl[q];
                }
#pragma unroll
            for (int q = 1; q < kAJ; ++q)
                if (q < nc) Mx[(q - 1) * ldv + i] = v[q] - 2.0 * p * hl[q];
        }
    }
}

__global__ void k_afinal(AdaptState* st, const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    st->r = st->r_new;
}

__global__ void k_areset(AdaptState* st) {
    st->r = 0;
    st->ok = 0;
    st->remove = 0;
    st->r_old = st->r_new = 0;
    st->mu = 0.0;
    st->nu = 0.0;
}

// ------------------------------------------------------------------ host
static int small_grid(const EngineArgs& e) { return e.NB; }

// U and A U at full size (2 (r_max + 1) columns of 8N bytes) take more than
// half of the 256 MiB last-level cache: the per-step operator streams them.
static bool stream_u(const EngineArgs& e) {
    return 2.0 * (e.adapt->rmax + 1) * 8.0 * (double)e.n > 128.0 * 1024.0 * 1024.0;
}

void adapt_reset(hipStream_t st, const AdaptArgs& a) { k_areset<<<1, 1, 0, st>>>(a.st); }

// s = C U^T (scale * x) for the SpMV input x of the step (gate 2).
void adapt_pre(const EngineArgs& e, const double* x, const double* scale) {
    const AdaptArgs& a = *e.adapt;
    const int NB = small_grid(e);
    if (stream_u(e))
        k_udots<true><<<NB, kWG, 0, e.st>>>(e.n, e.ldv, a.U, a.st, 1, nullptr, x, scale, a.part, NB,
                                            e.ctrl, 2);
    else
        k_udots<false><<<NB, kWG, 0, e.st>>>(e.n, e.ldv, a.U, a.st, 1, nullptr, x, scale, a.part, NB,
                                             e.ctrl, 2);
    k_ucoef<<<1, kUC, 0, e.st>>>(a.st, 1, 0, a.part, NB, a.C, a.rmax + 1, a.s, nullptr, e.ctrl, 2);
}

// y += (A U) s (gate 2).
void adapt_post(const EngineArgs& e, double* y) {
    const AdaptArgs& a = *e.adapt;
    if (stream_u(e))
        k_ucorr<true><<<small_grid(e), kWG, 0, e.st>>>(e.n, e.ldv, a.AU, a.st, a.s, 1.0, y, e.ctrl, 2);
    else
        k_ucorr<false><<<small_grid(e), kWG, 0, e.st>>>(e.n, e.ldv, a.AU, a.st, a.s, 1.0, y, e.ctrl, 2);
}

static void spmv_into(const EngineArgs& e, const double* x, double* y) {
    if (e.L == kSell)
        launch_spmv_sell_f64(e.st, e.NB, e.n, e.sell_off, e.sell_perm, e.sell_wuni, e.sell_wmax,
                             e.sell_col,
                             reinterpret_cast<const double*>(e.sell_val), x, y);
    else
        launch_spmv_f64(e.st, e.L, e.NB, e.n, e.rowptr, e.colind,
                        reinterpret_cast<const double*>(e.vals), x, y);
}

// End of a cycle (gate 1): x += M^{-1} (V_k y_k), then the update of U, AU, T
// and C from this cycle's Hessenberg matrix and basis.
void adapt_cycle_end(const EngineArgs& e, const double* V, const double* coef) {
    const AdaptArgs& a = *e.adapt;
    const int NB = small_grid(e);
    const int ld = a.rmax + 1;
    hipStream_t st = e.st;
    // x += d + U C U^T d,  d = V_k y_k
    k_vcomb<<<NB, kWG, 0, st>>>(e.n, e.ldv, V, coef, a.dvec, e.ctrl, 1);
    k_udots<false><<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.st, 1, nullptr, a.dvec, nullptr, a.part, NB, e.ctrl, 1);
    k_ucoef<<<1, kUC, 0, st>>>(a.st, 1, 0, a.part, NB, a.C, ld, a.s, nullptr, e.ctrl, 1);
    k_uaxpy<<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.st, a.s, a.dvec, e.xh, e.ctrl, 1);
    // Ritz vector u = V_k z of the smallest eigenvalue of H_k, |mu|.
    k_ritz<<<1, kSW, 0, st>>>(e.m, e.Hraw, e.vscale, a.st, a.zc, e.ctrl, 1);
    k_vcomb<<<NB, kWG, 0, st>>>(e.n, e.ldv, V, a.zc, a.ucand, e.ctrl, 1);
    // Classical Gram-Schmidt against U, twice.
    for (int pass = 0; pass < 2; ++pass) {
        k_udots<false><<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.st, 1, nullptr, a.ucand, nullptr, a.part, NB, e.ctrl, 1);
        k_ucoef<<<1, kUC, 0, st>>>(a.st, 1, 0, a.part, NB, nullptr, 0, a.s, nullptr, e.ctrl, 1);
        k_ucorr<false><<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.st, a.s, -1.0, a.ucand, e.ctrl, 1);
    }
    k_udots<false><<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.st, 0, a.ucand, a.ucand, nullptr, a.part, NB, e.ctrl, 1);
    k_unorm<<<1, kWG, 0, st>>>(a.part, NB, a.st, e.ctrl, 1);
    k_uscale<<<NB, kWG, 0, st>>>(e.n, a.ucand, a.st, e.ctrl, 1);
    spmv_into(e, a.ucand, a.aucand);
    // New column of T: U_q . A u (q < r) and u . A u; new row: u . A U_q.
    k_udots<false><<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.st, 1, a.ucand, a.aucand, nullptr, a.part, NB, e.ctrl, 1);
    k_ucoef<<<1, kUC, 0, st>>>(a.st, 1, 1, a.part, NB, nullptr, 0, a.s, a.tcol, e.ctrl, 1);
    k_udots<false><<<NB, kWG, 0, st>>>(e.n, e.ldv, a.AU, a.st, 1, nullptr, a.ucand, nullptr, a.part, NB, e.ctrl, 1);
    k_ucoef<<<1, kUC, 0, st>>>(a.st, 1, 0, a.part, NB, nullptr, 0, a.s, a.trow, e.ctrl, 1);
    k_tupdate<<<1, kSW, 0, st>>>(a.rmax, a.T, a.C, a.tcol, a.trow, a.hvec, a.st, e.ctrl, 1);
    k_ucommit<<<NB, kWG, 0, st>>>(e.ldv, a.U, a.AU, a.ucand, a.aucand, a.st, e.ctrl, 1);
    k_householder<<<NB, kWG, 0, st>>>(e.n, e.ldv, a.U, a.AU, a.hvec, a.st, e.ctrl, 1);
    k_afinal<<<1, 1, 0, st>>>(a.st, e.ctrl, 1);
}

GM_DEBUG_ACCESSOR(dbg_take_adapt)

}  // namespace gm
