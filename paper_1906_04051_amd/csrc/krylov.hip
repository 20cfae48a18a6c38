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
#include "internal.hpp"

namespace gm {

__device__ __forceinline__ bool gated(const Ctrl* c, int gate) {
    if (gate == 0 || c == nullptr) return false;
    return c->done != 0 || (gate == 2 && c->stop != 0);
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
        for (int k = k0 + lane; k < k1; k += L) s += (ACC)vals[k] * (ACC)ld_f(x + colind[k]);
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
        if (lane == 0) y[row] = (YT)(s * scale);
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

// s = E^{-1} t with t = sum over chunks of tpart (fixed order).  Einv is the
// explicit inverse of E built from its LU factors at setup, column-major
// (Einv[i][a] at Einv[a*R + i]); `trans` applies E^{-T} instead (adjoint).
__global__ __launch_bounds__(kWG) void k_coarse(int R, int MC, const double* __restrict__ tpart,
                                                const double* __restrict__ Einv, int trans,
                                                double* __restrict__ s, const Ctrl* ctrl,
                                                int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ double t[kMaxR];
    for (int a = threadIdx.x; a < R; a += kWG) {
        double acc = 0;
        for (int c = 0; c < MC; ++c) acc += tpart[(int64_t)a * MC + c];
        t[a] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += kWG) {
        double acc = 0;
        if (!trans)
            for (int a = 0; a < R; ++a) acc += Einv[(int64_t)a * R + i] * t[a];
        else
            for (int a = 0; a < R; ++a) acc += Einv[(int64_t)i * R + a] * t[a];
        s[i] = acc;
    }
}

// ------------------------------------------------------------- CGS2 passes
// Lane layout: T consecutive lanes share one row; lane `sub` of the group owns
// basis columns k = sub, sub + T, sub + 2T, ... so each lane keeps JMAX / T
// basis entries and dot accumulators in registers.

// Sum over the T lanes of a row group (butterfly; same value in all of them).
template <int T, typename ACC>
__device__ __forceinline__ ACC group_sum(ACC v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
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
                                               const double* __restrict__ s, int R,
                                               WT* __restrict__ w, double* __restrict__ part,
                                               int nslot, int NB, const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    constexpr int JT = JMAX / T;
    __shared__ ACC s_l[kMaxR];
    __shared__ ACC red[kWG / kWave][JMAX + 1];
    for (int a = threadIdx.x; a < R; a += kWG) s_l[a] = (ACC)s[a];
    __syncthreads();
    const int sub = threadIdx.x & (T - 1);
    ACC acc[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) acc[q] = 0;
    ACC accn = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T);
    for (int64_t i = ((int64_t)blockIdx.x * kWG + threadIdx.x) / T; i < n; i += stride) {
        ACC wi = (ACC)y[i];
        if (R > 0)
            for (int q = azrp[i]; q < azrp[i + 1]; ++q) wi -= (ACC)azv[q] * s_l[azci[q]];
        if (sub == 0) {
            w[i] = (WT)wi;
            accn += wi * wi;
        }
        ACC vv[JT];
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) vv[q] = (ACC)ld_f(V + (sub + q * T) * ldv + i);
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) acc[q] += vv[q] * wi;
    }
    store_partials<JMAX, T, ACC>(acc, accn, nv, red, part, nslot, NB);
}

// Pass 2: w -= sum_k stored_k c_k (first Gram-Schmidt update), then partial
// dots stored_k^T w and ||w||^2 of the updated vector.
template <int JMAX, int T, typename VT, typename WT, typename ACC>
__global__ __launch_bounds__(kWG) void k_pass2(int n, int64_t ldv, const VT* __restrict__ V, int nv,
                                               WT* __restrict__ w, const double* __restrict__ coef,
                                               double* __restrict__ part, int nslot, int NB,
                                               const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    constexpr int JT = JMAX / T;
    __shared__ ACC c_l[JMAX];
    __shared__ ACC red[kWG / kWave][JMAX + 1];
    for (int k = threadIdx.x; k < nv; k += kWG) c_l[k] = (ACC)coef[k];
    __syncthreads();
    const int sub = threadIdx.x & (T - 1);
    ACC acc[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) acc[q] = 0;
    ACC accn = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T);
    for (int64_t i = ((int64_t)blockIdx.x * kWG + threadIdx.x) / T; i < n; i += stride) {
        ACC vv[JT];
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) vv[q] = (ACC)ld_f(V + (sub + q * T) * ldv + i);
        ACC u = 0;
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) u += vv[q] * c_l[sub + q * T];
        const ACC wi = (ACC)w[i] - group_sum<T>(u);
        if (sub == 0) {
            w[i] = (WT)wi;
            accn += wi * wi;
        }
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) acc[q] += vv[q] * wi;
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
                                               const Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    constexpr int JT = JMAX / T;
    __shared__ ACC c_l[JMAX];
    __shared__ ACC red[kWG / kWave];
    for (int k = threadIdx.x; k < nv; k += kWG) c_l[k] = (ACC)coef[k];
    __syncthreads();
    const ACC sg = (ACC)(*sigma);
    VT* __restrict__ vout = V + nv * ldv;
    const int sub = threadIdx.x & (T - 1);
    ACC accn = 0;
    const int64_t stride = (int64_t)gridDim.x * (kWG / T);
    for (int64_t i = ((int64_t)blockIdx.x * kWG + threadIdx.x) / T; i < n; i += stride) {
        ACC vv[JT];
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) vv[q] = (ACC)ld_f(V + (sub + q * T) * ldv + i);
        ACC u = 0;
#pragma unroll
        for (int q = 0; q < JT; ++q)
            if (sub + q * T < nv) u += vv[q] * c_l[sub + q * T];
        const ACC wi = (ACC)w[i] - group_sum<T>(u);
        if (sub == 0) {
            st_v(vout + i, wi * sg);
            accn += wi * wi;
        }
    }
    const ACC t = block_sum(accn, red);
    if (threadIdx.x == 0) part[(int64_t)nslot * NB + blockIdx.x] = (double)t;
}

// Finish the partial sums of one pass (one workgroup per slot, fixed order).
// Slots k < nv: h[k] = vscale[k] * sum (Hessenberg entries against the
// normalised v_k) and coef[k] = h[k] * vscale[k] (coefficient of stored_k).
// The norm slot: mode 1 writes ||w||^2 to ctrl->wpre2 (breakdown reference);
// mode 2 sets the storage scale sigma (sqrt(N)/||w|| for FP16 storage, else 1).
__global__ __launch_bounds__(kWG) void k_finish(const double* __restrict__ part, int NB, int nv,
                                                int nslot, const double* __restrict__ vscale,
                                                double* __restrict__ h, double* __restrict__ coef,
                                                int mode, int half_store, double nscale,
                                                double* __restrict__ sigma, Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    __shared__ double red[kWG / kWave];
    const int b = blockIdx.x;
    const int slot = (b < nv) ? b : nslot;
    double acc = 0;
    for (int q = threadIdx.x; q < NB; q += kWG) acc += part[(int64_t)slot * NB + q];
    acc = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    if (b < nv) {
        const double hk = vscale[b] * acc;
        h[b] = hk;
        coef[b] = hk * vscale[b];
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
// (h_{j+1,j} <= eps * ||P A v_j||) or the iteration cap.
__global__ __launch_bounds__(kWave) void k_givens(int j, int m, const double* __restrict__ part,
                                                  int NB, int nslot, const double* __restrict__ h1,
                                                  const double* __restrict__ h2,
                                                  double* __restrict__ H, double* __restrict__ cs,
                                                  double* __restrict__ sn, double* __restrict__ g,
                                                  double* __restrict__ vscale,
                                                  const double* __restrict__ sigma,
                                                  double* __restrict__ hist, int64_t hist_cap,
                                                  double* __restrict__ Hraw, Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    double acc = 0;
    for (int q = threadIdx.x; q < NB; q += kWave) acc += part[(int64_t)nslot * NB + q];
    acc = wave_sum(acc);
    if (threadIdx.x != 0) return;
    const double hn = sqrt(acc);
    double col[kMaxM + 1];
    for (int k = 0; k <= j; ++k) col[k] = h1[k] + h2[k];
    col[j + 1] = hn;
    if (Hraw)
        for (int k = 0; k <= j + 1; ++k) Hraw[(int64_t)k * m + j] = col[k];
    const double wpre = sqrt(ctrl->wpre2);
    const int bd = !(hn > 2.220446049250313e-16 * wpre);
    for (int i = 0; i < j; ++i) {
        const double a = col[i], c = col[i + 1];
        col[i] = cs[i] * a + sn[i] * c;
        col[i + 1] = -sn[i] * a + cs[i] * c;
    }
    const double a = col[j], c = col[j + 1];
    double rho = hypot(a, c);
    if (c == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
        rho = a;
    } else {
        cs[j] = a / rho;
        sn[j] = c / rho;
    }
    col[j] = rho;
    col[j + 1] = 0.0;
    for (int k = 0; k <= j + 1; ++k) H[(int64_t)k * m + j] = col[k];
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    vscale[j + 1] = bd ? 0.0 : 1.0 / ((*sigma) * hn);
    const int64_t its = ctrl->its + 1;
    ctrl->its = its;
    if (hist && its - 1 < hist_cap) hist[its - 1] = fabs(g[j + 1]);
    ctrl->k = j + 1;
    ctrl->breakdown = bd;
    if (fabs(g[j + 1]) <= ctrl->target || bd || its >= ctrl->max_iters) ctrl->stop = 1;
}

// Back substitution R_k y = g_{1:k}; coef[i] = y_i * vscale[i] (coefficient of
// stored_i in x_hat += V_k y).
__global__ __launch_bounds__(kWave) void k_backsolve(int m, const double* __restrict__ H,
                                                     const double* __restrict__ g,
                                                     const double* __restrict__ vscale,
                                                     double* __restrict__ coef, int* cyc_k,
                                                     int cyc_cap, Ctrl* ctrl, int gate) {
    if (gated(ctrl, gate)) return;
    if (threadIdx.x != 0) return;
    const int k = ctrl->k;
    if (cyc_k && ctrl->cycles - 1 < cyc_cap) cyc_k[ctrl->cycles - 1] = k;
    double y[kMaxM];
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int q = i + 1; q < k; ++q) s -= H[(int64_t)i * m + q] * y[q];
        y[i] = s / H[(int64_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) coef[i] = y[i] * vscale[i];
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
                         double* __restrict__ vscale, double* __restrict__ sigma0, Ctrl* ctrl) {
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
    } else if (beta <= ctrl->target) {
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

__global__ void k_ctrl_reset(Ctrl* ctrl, int64_t max_iters) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctrl c = {};
        c.max_iters = max_iters;
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

template <typename AT, typename XT, typename YT, typename ACC>
static void spmv_dispatch(int L, int NB, hipStream_t st, int n, const int* rp, const int* ci,
                          const AT* v, const XT* x, const double* scale, YT* y, const Ctrl* c,
                          int gate) {
    dim3 g(NB), b(kWG);
    switch (L) {
        case 1: k_spmv<1, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
        case 2: k_spmv<2, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
        case 4: k_spmv<4, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
        case 8: k_spmv<8, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
        case 16: k_spmv<16, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
        case 32: k_spmv<32, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
        default: k_spmv<64, AT, XT, YT, ACC><<<g, b, 0, st>>>(n, rp, ci, v, x, scale, y, c, gate); break;
    }
}

template <typename AT, typename BT, typename RT, typename ACC>
static void residual_dispatch(int L, int NB, hipStream_t st, int n, const int* rp, const int* ci,
                              const AT* v, const double* x, const BT* b, RT* r, double* part,
                              int slot, const Ctrl* c, int gate) {
    dim3 g(NB), bl(kWG);
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

static int jmax_for(int nv) {
    if (nv <= 8) return 8;
    if (nv <= 16) return 16;
    if (nv <= 32) return 32;
    if (nv <= 48) return 48;
    if (nv <= 64) return 64;
    return 96;
}

// Lanes per row of the pass kernels: keep JMAX / T register entries per lane
// at or below 24 (FP64) / 48 (FP32) so no instantiation spills.
template <int J, typename ACC>
struct LanesFor {
    static constexpr int kCap = sizeof(ACC) == 8 ? 24 : 48;
    static constexpr int value = J <= kCap ? 1 : (J <= 2 * kCap ? 2 : 4);
};

#define GM_JMAX_SWITCH(nv, ACCT, CALL)                                                         \
    switch (jmax_for(nv)) {                                                                    \
        case 8: { constexpr int J = 8; constexpr int T = LanesFor<J, ACCT>::value; CALL; } break;   \
        case 16: { constexpr int J = 16; constexpr int T = LanesFor<J, ACCT>::value; CALL; } break; \
        case 32: { constexpr int J = 32; constexpr int T = LanesFor<J, ACCT>::value; CALL; } break; \
        case 48: { constexpr int J = 48; constexpr int T = LanesFor<J, ACCT>::value; CALL; } break; \
        case 64: { constexpr int J = 64; constexpr int T = LanesFor<J, ACCT>::value; CALL; } break; \
        default: { constexpr int J = 96; constexpr int T = LanesFor<J, ACCT>::value; CALL; } break; \
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
    static constexpr int kHalf = std::is_same<VT, __half>::value ? 1 : 0;

    void coarse(const WT* vec, double* s, int gate) const {
        if (e.R == 0) return;
        k_zt<WT><<<e.R * e.MC, kWG, 0, e.st>>>(e.R, e.MC, e.CH, e.ztrp, e.ztci, e.ztv, vec, e.tpart,
                                              e.ctrl, gate);
        k_coarse<<<1, kWG, 0, e.st>>>(e.R, e.MC, e.tpart, e.Einv, e.trans, s, e.ctrl, gate);
    }

    // Residual of x_hat, its deflated version p = P r into e.p, and the
    // restart decision (or the initialisation when `init`).
    template <typename BT>
    void restart_block(const BT* b, bool init, double rtol, double r0_override) const {
        residual_dispatch<AT, BT, WT, ACC>(e.L, e.NB, e.st, e.n, e.rowptr, e.colind, vals(), e.xh, b,
                                           r(), e.part, e.nslot, e.ctrl, init ? 0 : 1);
        if (init) k_init<<<1, kWG, 0, e.st>>>(e.part, e.NB, e.nslot, rtol, r0_override, e.ctrl);
        coarse(r(), e.s_res, init ? 0 : 1);
        k_pass1<8, 1, VT, WT, AT, ACC><<<e.NB, kWG, 0, e.st>>>(e.n, e.ldv, V(), 0, r(), e.azrp, e.azci,
                                                            azv(), e.s_res, e.R, p(), e.part,
                                                            e.nslot, e.NB, e.ctrl, 1);
        k_decide<<<1, kWG, 0, e.st>>>(e.part, e.NB, e.nslot, e.m, kHalf, e.nscale, e.g, e.vscale,
                                      e.sigma0, e.ctrl);
        k_store_v0<VT, WT><<<e.NB, kWG, 0, e.st>>>(e.n, p(), e.sigma0, Vcol(0), e.ctrl, 1);
    }

    void step(int j) const {
        const int nv = j + 1;
        if (e.timer) e.timer->begin(0, j);
        spmv_dispatch<AT, VT, WT, ACC>(e.L, e.NB, e.st, e.n, e.rowptr, e.colind, vals(), Vcol(j),
                                       e.vscale + j, y(), e.ctrl, 2);
        if (e.timer) e.timer->end(0, j);
        coarse(y(), e.s_step, 2);
        if (e.timer) e.timer->begin(1, j);
        GM_JMAX_SWITCH(nv, ACC, (k_pass1<J, T, VT, WT, AT, ACC><<<e.NB, kWG, 0, e.st>>>(
                               e.n, e.ldv, V(), nv, y(), e.azrp, e.azci, azv(), e.s_step, e.R, w(),
                               e.part, e.nslot, e.NB, e.ctrl, 2)));
        if (e.timer) e.timer->end(1, j);
        k_finish<<<nv + 1, kWG, 0, e.st>>>(e.part, e.NB, nv, e.nslot, e.vscale, e.h1, e.coef1, 1,
                                           kHalf, e.nscale, e.sigma, e.ctrl, 2);
        if (e.timer) e.timer->begin(2, j);
        GM_JMAX_SWITCH(nv, ACC, (k_pass2<J, T, VT, WT, ACC><<<e.NB, kWG, 0, e.st>>>(
                               e.n, e.ldv, V(), nv, w(), e.coef1, e.part, e.nslot, e.NB, e.ctrl, 2)));
        if (e.timer) e.timer->end(2, j);
        k_finish<<<nv + 1, kWG, 0, e.st>>>(e.part, e.NB, nv, e.nslot, e.vscale, e.h2, e.coef2, 2,
                                           kHalf, e.nscale, e.sigma, e.ctrl, 2);
        if (e.timer) e.timer->begin(3, j);
        GM_JMAX_SWITCH(nv, ACC, (k_pass3<J, T, VT, WT, ACC><<<e.NB, kWG, 0, e.st>>>(
                               e.n, e.ldv, V(), nv, w(), e.coef2, e.sigma, e.part, e.nslot, e.NB,
                               e.ctrl, 2)));
        if (e.timer) e.timer->end(3, j);
        k_givens<<<1, kWave, 0, e.st>>>(j, e.m, e.part, e.NB, e.nslot, e.h1, e.h2, e.H, e.cs, e.sn,
                                        e.g, e.vscale, e.sigma, e.hist, e.hist_cap, e.Hraw, e.ctrl, 2);
    }

    template <typename BT>
    void cycle(const BT* b) const {
        for (int j = 0; j < e.m; ++j) step(j);
        k_backsolve<<<1, kWave, 0, e.st>>>(e.m, e.H, e.g, e.vscale, e.coef1, e.cyc_k, e.cyc_cap,
                                           e.ctrl, 1);
        k_xupdate<VT><<<e.NB, kWG, 0, e.st>>>(e.n, e.ldv, V(), e.coef1, e.xh, e.ctrl, 1);
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

void launch_pass_probe(const EngineArgs& e, int kind, int nv) {
    using VT = double;
    using WT = double;
    using ACC = double;
    using AT = double;
    const VT* V = reinterpret_cast<const VT*>(e.V);
    WT* y = reinterpret_cast<WT*>(e.y);
    WT* w = reinterpret_cast<WT*>(e.w);
    if (kind == 1) {
        GM_JMAX_SWITCH(nv, ACC, (k_pass1<J, T, VT, WT, AT, ACC><<<e.NB, kWG, 0, e.st>>>(
                                    e.n, e.ldv, V, nv, y, e.azrp, e.azci, (const AT*)e.azv, e.s_step,
                                    e.R, w, e.part, e.nslot, e.NB, nullptr, 0)));
    } else if (kind == 2) {
        GM_JMAX_SWITCH(nv, ACC, (k_pass2<J, T, VT, WT, ACC><<<e.NB, kWG, 0, e.st>>>(
                                    e.n, e.ldv, V, nv, w, e.coef1, e.part, e.nslot, e.NB, nullptr, 0)));
    } else {
        GM_JMAX_SWITCH(nv, ACC, (k_pass3<J, T, VT, WT, ACC><<<e.NB, kWG, 0, e.st>>>(
                                    e.n, e.ldv, (VT*)V, nv, w, e.coef2, e.sigma, e.part, e.nslot,
                                    e.NB, nullptr, 0)));
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

void launch_ctrl_reset(hipStream_t st, Ctrl* c, int64_t max_iters) {
    k_ctrl_reset<<<1, 64, 0, st>>>(c, max_iters);
}

void launch_fill(hipStream_t st, double* p, int64_t n, double v) {
    const int64_t nb = std::min<int64_t>((n + kWG - 1) / kWG, 2048);
    if (nb > 0) k_fill<<<(int)nb, kWG, 0, st>>>(p, n, v);
}

void launch_copy(hipStream_t st, const double* a, double* b, int64_t n) {
    const int64_t nb = std::min<int64_t>((n + kWG - 1) / kWG, 2048);
    if (nb > 0) k_copy_f64<<<(int)nb, kWG, 0, st>>>(a, b, n);
}

}  // namespace gm
